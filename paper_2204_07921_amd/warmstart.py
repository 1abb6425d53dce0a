"""Learned warm start for the multigrid solver.

The network (libmgcurv.so, mg_cnn_*) is trained on pairs (f, u*) in which u* is what the
batched multigrid solver itself returns for f (mean curvature, alpha 20, stop at a relative
energy change of 1e-6).  At solve time u0 = f + g(f) replaces u0 = f, and the multigrid
refines u0 until its energy reaches the plain solve's final energy F_plain (1 + 1e-6); an image
whose warm-started refinement does not get there within the V-cycle budget falls back to the
plain solve from u0 = f, whose time is then counted too.  The plain solve's energy remains the
reference the final energy is held to.

    python -m paper_2204_07921_amd.warmstart train --pairs 20000 --size 256 --steps 3000 --out W.npz
    python -m paper_2204_07921_amd.warmstart eval --weights W.npz --n 64 --size 1024
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import mgcurv

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "warmstart_mean_alpha20.npz")
ALPHA = 20.0
KIND = mgcurv.MG_CURV_MEAN


def _log(msg: str):
    print(msg, file=sys.stderr, flush=True)


def make_inputs(n: int, size: int, seed0: int) -> torch.Tensor:
    """n seeded noisy images (size x size, sigma ~ U[0.03, 0.12]) as a float32 device tensor."""
    from synth import noisy_image
    rng = np.random.Generator(np.random.PCG64(seed0))
    sig = rng.uniform(0.03, 0.12, size=n)
    out = torch.empty(n, size, size, dtype=torch.float32, device="cuda")
    for i in range(n):
        f, _ = noisy_image(size, size, seed0 + i, float(sig[i]), dtype=np.float32)
        out[i].copy_(torch.from_numpy(f))
    return out


def solve_batch(f: torch.Tensor, u0: torch.Tensor | None = None, rel_tol: float = 1e-6, max_vcycles: int = 300,
                targets=None, tune: bool = True):
    """Solve a stack of equally sized images with the batched path; returns (u, result dict)."""
    n, h, w = f.shape
    bs = mgcurv.BatchSolver([dict(height=h, width=w, alpha=ALPHA, kind=KIND)] * n)
    fd = f.reshape(-1).contiguous()
    ud = (f if u0 is None else u0).reshape(-1).clone()
    if tune:
        bs.tune(ud, fd, repeats=1)
    if targets is None:
        res = bs.solve(ud, fd, rel_tol=rel_tol, max_vcycles=max_vcycles)
    else:
        res = bs.solve_target(ud, fd, targets, max_vcycles=max_vcycles)
    bs.close()
    return ud.view(n, h, w), res


def make_pairs(n_pairs: int, size: int, seed0: int = 0, chunk: int = 1024, max_vcycles: int = 300):
    """Training pairs (f, u*) on the device; u* from the batched multigrid solver."""
    fs, us = [], []
    t0 = time.perf_counter()
    for start in range(0, n_pairs, chunk):
        m = min(chunk, n_pairs - start)
        f = make_inputs(m, size, seed0 + start)
        u, res = solve_batch(f, max_vcycles=max_vcycles)
        fs.append(f)
        us.append(u)
        _log(f"pairs {start + m}/{n_pairs}: mean V-cycles {np.mean(res['vcycles']):.1f}, "
             f"{time.perf_counter() - t0:.1f} s")
    return torch.cat(fs), torch.cat(us)


def train(net: mgcurv.WarmStartCNN, f: torch.Tensor, u: torch.Tensor, steps: int, batch: int,
          lr_max: float = 2e-3, lr_min: float = 2e-5, seed: int = 0, log_every: int = 250):
    """Adam on minibatches drawn by a seeded permutation; cosine learning-rate decay."""
    g = torch.Generator().manual_seed(seed)
    n = f.shape[0]
    order = torch.randperm(n, generator=g)
    pos = 0
    losses = []
    for s in range(steps):
        if pos + batch > n:
            order = torch.randperm(n, generator=g)
            pos = 0
        idx = order[pos:pos + batch].cuda()
        pos += batch
        lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + np.cos(np.pi * s / max(1, steps - 1)))
        fb = f.index_select(0, idx).contiguous()
        ub = u.index_select(0, idx).contiguous()
        want = (s % log_every == 0) or s == steps - 1
        loss = net.train_step(fb, ub, lr, want_loss=want)
        if want:
            losses.append((s, loss))
            _log(f"step {s}: loss {loss:.4e} lr {lr:.2e}")
    return losses


def forward_chunked(net: mgcurv.WarmStartCNN, f: torch.Tensor) -> torch.Tensor:
    n, h, w = f.shape
    per = max(1, net.max_pixels // (h * w))
    out = torch.empty_like(f)
    for s in range(0, n, per):
        net.forward(f[s:s + per].contiguous(), out[s:s + per])
    return out


def evaluate(net: mgcurv.WarmStartCNN, f: torch.Tensor, rel_tol: float = 1e-6, budget_factor: float = 3.0,
             max_vcycles: int = 1000) -> dict:
    """Plain batched solve from u0 = f against the warm-started one (CNN time included)."""
    torch.cuda.synchronize()
    t = time.perf_counter()
    u_plain, rp = solve_batch(f, rel_tol=rel_tol, max_vcycles=max_vcycles, tune=False)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    e_plain = np.array(rp["energy"])
    targets = e_plain * (1 + 1e-6)
    budget = int(budget_factor * max(rp["vcycles"])) + 1
    torch.cuda.synchronize()
    t = time.perf_counter()
    u0 = forward_chunked(net, f)
    torch.cuda.synchronize()
    t_cnn = time.perf_counter() - t
    u_warm, rw = solve_batch(f, u0=u0, targets=targets, max_vcycles=budget, tune=False)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t
    missed = [i for i, s in enumerate(rw["image_status"]) if s != 0]
    t_fallback = 0.0
    if missed:
        t = time.perf_counter()
        solve_batch(f[missed].contiguous(), rel_tol=rel_tol, max_vcycles=max_vcycles, tune=False)
        torch.cuda.synchronize()
        t_fallback = time.perf_counter() - t
    e_warm = np.array(rw["energy"])
    # second protocol: refine the CNN prediction with the plain stopping rule itself
    torch.cuda.synchronize()
    t = time.perf_counter()
    u0b = forward_chunked(net, f)
    _, rt = solve_batch(f, u0=u0b, rel_tol=rel_tol, max_vcycles=max_vcycles, tune=False)
    torch.cuda.synchronize()
    t_tol = time.perf_counter() - t
    e_tol = np.array(rt["energy"])
    return {"images": int(f.shape[0]), "size": list(f.shape[1:]),
            "plain": {"seconds": round(t_plain, 4), "vcycles_mean": float(np.mean(rp["vcycles"])),
                      "vcycles_max": int(max(rp["vcycles"])), "converged": int(sum(s == 0 for s in rp["image_status"]))},
            "warm": {"seconds": round(t_warm + t_fallback, 4), "cnn_seconds": round(t_cnn, 4),
                     "refine_seconds": round(t_warm - t_cnn, 4), "fallback_seconds": round(t_fallback, 4),
                     "vcycles_mean": float(np.mean(rw["vcycles"])), "vcycles_max": int(max(rw["vcycles"])),
                     "reached_plain_energy": int(len(e_warm) - len(missed)), "fallbacks": len(missed)},
            "vcycles_saved_mean": float(np.mean(rp["vcycles"]) - np.mean(rw["vcycles"])),
            "final_energy_gap_rel_max": float(np.max((e_warm - e_plain) / e_plain)),
            "final_energy_gap_rel_mean": float(np.mean((e_warm - e_plain) / e_plain)),
            "speedup": round(t_plain / max(1e-9, t_warm + t_fallback), 3),
            "warm_to_stopping_rule": {"seconds": round(t_tol, 4), "vcycles_mean": float(np.mean(rt["vcycles"])),
                                      "vcycles_max": int(max(rt["vcycles"])),
                                      "energy_gap_rel_mean": float(np.mean((e_tol - e_plain) / e_plain))}}


def evaluate_single(net: mgcurv.WarmStartCNN, f: torch.Tensor, fine_colours: int = 9, rel_tol: float = 1e-6,
                    budget_factor: float = 3.0, max_vcycles: int = 2000) -> dict:
    """The same comparison image by image on the single-image solver, which also runs the nine-colour
    pixel level (the batched path runs four colours only).  Per image: the plain solve from u0 = f to
    the relative energy change rel_tol gives F_plain; the warm start (CNN forward, then V-cycles until
    F <= F_plain (1 + 1e-6), within budget_factor x the plain V-cycles, else the plain solve as
    fallback, its time added) is timed CNN included."""
    n, h, w = f.shape
    s = mgcurv.Solver(h, w, alpha=ALPHA, kind=KIND, dtype=torch.float32, fine_colours=fine_colours)
    u = f[0].clone()
    s.vcycle(u, f[0].contiguous())   # warm-up
    forward_chunked(net, f[:1].contiguous())
    rows = []
    for k in range(n):
        fk = f[k].contiguous()
        u = fk.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        rp = s.solve(u, fk, rel_tol=rel_tol, max_vcycles=max_vcycles)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t
        t = time.perf_counter()
        u0 = forward_chunked(net, f[k:k + 1].contiguous())[0]
        torch.cuda.synchronize()
        t_cnn = time.perf_counter() - t
        e_cnn = s.energy(u0, fk)
        t = time.perf_counter()
        rw = s.solve_target(u0, fk, rp["energy"] * (1 + 1e-6), max_vcycles=int(budget_factor * rp["vcycles"]) + 1)
        torch.cuda.synchronize()
        t_warm = t_cnn + time.perf_counter() - t
        fallback = rw["status"] != 0
        if fallback:
            uu = fk.clone()
            t = time.perf_counter()
            s.solve(uu, fk, rel_tol=rel_tol, max_vcycles=max_vcycles)
            torch.cuda.synchronize()
            t_warm += time.perf_counter() - t
        rows.append({"plain_vcycles": rp["vcycles"], "plain_status": rp["status"], "plain_energy": rp["energy"],
                     "plain_seconds": t_plain, "cnn_energy": e_cnn, "warm_vcycles": rw["vcycles"],
                     "warm_energy": rw["energy"], "warm_seconds": t_warm, "fallback": fallback})
    s.close()
    tp = sum(r["plain_seconds"] for r in rows)
    tw = sum(r["warm_seconds"] for r in rows)
    return {"images": n, "size": [h, w], "fine_colours": fine_colours,
            "plain": {"seconds": round(tp, 4), "vcycles_mean": float(np.mean([r["plain_vcycles"] for r in rows])),
                      "converged": int(sum(r["plain_status"] == 0 for r in rows))},
            "cnn_above_plain_energy": int(sum(r["cnn_energy"] > r["plain_energy"] for r in rows)),
            "warm": {"seconds": round(tw, 4), "vcycles_mean": float(np.mean([r["warm_vcycles"] for r in rows])),
                     "vcycles_min": int(min(r["warm_vcycles"] for r in rows)),
                     "vcycles_max": int(max(r["warm_vcycles"] for r in rows)),
                     "fallbacks": int(sum(r["fallback"] for r in rows))},
            "final_energy_gap_rel_max": float(max((r["warm_energy"] - r["plain_energy"]) / r["plain_energy"] for r in rows)),
            "speedup": round(tp / max(tw, 1e-9), 3), "per_image": rows}


def save(path: str, params: np.ndarray, meta: dict):
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(params, dtype=np.float32), meta=json.dumps(meta))


def save_checkpoint(path: str, state: dict, meta: dict | None = None):
    """Training checkpoint (parameters, Adam moments and step) as a plain .npz (no pickled objects)."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=np.asarray(state["params"], dtype=np.float32), m=np.asarray(state["m"], dtype=np.float32),
             v=np.asarray(state["v"], dtype=np.float32), step=np.int64(state["step"]), meta=json.dumps(meta or {}))


def load_checkpoint(path: str) -> dict:
    with np.load(path, allow_pickle=False) as z:
        return {"params": z["params"].astype(np.float32), "m": z["m"].astype(np.float32),
                "v": z["v"].astype(np.float32), "step": int(z["step"]), "meta": json.loads(str(z["meta"]))}


def load(path: str = DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["params"].astype(np.float32), json.loads(str(z["meta"]))


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    tr = sub.add_parser("train")
    tr.add_argument("--pairs", type=int, default=20000)
    tr.add_argument("--size", type=int, default=256)
    tr.add_argument("--steps", type=int, default=3000)
    tr.add_argument("--batch", type=int, default=16)
    tr.add_argument("--seed", type=int, default=0)
    tr.add_argument("--out", default=DEFAULT_WEIGHTS)
    tr.add_argument("--eval-n", type=int, default=0)
    tr.add_argument("--eval-size", type=int, default=1024)
    ev = sub.add_parser("eval")
    ev.add_argument("--weights", default=DEFAULT_WEIGHTS)
    ev.add_argument("--n", type=int, default=64)
    ev.add_argument("--size", type=int, default=1024)
    args = ap.parse_args()
    from synth import init_params
    if args.cmd == "train":
        t0 = time.perf_counter()
        f, u = make_pairs(args.pairs, args.size, seed0=args.seed)
        t_pairs = time.perf_counter() - t0
        net = mgcurv.WarmStartCNN(args.batch * args.size * args.size, init_params(args.seed))
        t1 = time.perf_counter()
        losses = train(net, f, u, args.steps, args.batch, seed=args.seed)
        torch.cuda.synchronize()
        t_train = time.perf_counter() - t1
        meta = {"pairs": args.pairs, "size": args.size, "steps": args.steps, "batch": args.batch,
                "seed": args.seed, "alpha": ALPHA, "kind": "mean", "pairs_seconds": round(t_pairs, 2),
                "train_seconds": round(t_train, 2), "losses": losses}
        save(args.out, net.get_params(), meta)
        _log(f"saved {args.out}")
        del f, u
        torch.cuda.empty_cache()
        if args.eval_n:
            fe = make_inputs(args.eval_n, args.eval_size, seed0=100000)
            net2 = mgcurv.WarmStartCNN(8 * args.eval_size * args.eval_size, net.get_params())
            meta["eval"] = evaluate(net2, fe)
            save(args.out, net.get_params(), meta)
        print(json.dumps(meta), flush=True)
    else:
        params, meta = load(args.weights)
        fe = make_inputs(args.n, args.size, seed0=100000)
        net = mgcurv.WarmStartCNN(8 * args.size * args.size, params)
        print(json.dumps(evaluate(net, fe)), flush=True)


if __name__ == "__main__":
    main()
