"""Level-count, cycle-shape and size study of the paper's own local step (Section 4, the
experiments behind Tables 2-3): for synthetic images in the paper's intensity regime it
solves to relErr(u) < 1e-4 with J = 1..6 levels, half (fine to coarse) and full
(fine-coarse-fine) V-cycles, and image sides 256..4096, and reports V-cycles, GPU time,
energy and RMSE to the clean image.

    python -m paper_2204_07921_amd.fbs_study [--sizes 256 512 1024 2048 4096] [--kind 0]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import mgcurv


def _image(n: int, seed: int):
    from synth import noisy_image
    f, g = noisy_image(n, n, seed, 0.08, dtype=np.float32)
    return (255.0 * f).astype(np.float32), 255.0 * g.astype(np.float64)


def run_case(f: torch.Tensor, g: np.ndarray, kind: int, levels: int, cycle: int, alpha: float,
             tol: float = 1e-4, max_vcycles: int = 500) -> dict:
    n = f.shape[0]
    s = mgcurv.FbsSolver(n, n, alpha=alpha, kind=kind, levels=levels, dtype=torch.float32, cycle=cycle)
    u = f.clone()
    s.solve(u, f, tol=tol, max_vcycles=1, stop=mgcurv.MG_STOP_RELERR_U)   # capture and warm up
    u = f.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = s.solve(u, f, tol=tol, max_vcycles=max_vcycles, stop=mgcurv.MG_STOP_RELERR_U)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    rmse = float(np.sqrt(np.mean((u.cpu().numpy().astype(np.float64) - g) ** 2)))
    s.close()
    return {"size": n, "levels": levels, "cycle": "full" if cycle else "half", "vcycles": res["vcycles"],
            "converged": res["status"] == 0, "seconds": round(el, 5),
            "ms_per_vcycle": round(el / max(1, res["vcycles"]) * 1e3, 4), "energy": res["energy"],
            "rmse": round(rmse, 4)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[256, 512, 1024, 2048, 4096])
    ap.add_argument("--kind", type=int, default=0)
    ap.add_argument("--alpha", type=float, default=0.05)
    ap.add_argument("--levels", type=int, nargs="+", default=[1, 2, 3, 4, 5, 6])
    args = ap.parse_args()
    rows = []
    f1, g1 = _image(1024, 7)
    fd = torch.tensor(f1, device="cuda")
    for cycle in (0, 1):
        for J in args.levels:
            r = run_case(fd, g1, args.kind, J, cycle, args.alpha)
            rows.append(r)
            print(json.dumps(r), file=sys.stderr, flush=True)
    for n in args.sizes:
        f, g = _image(n, 7)
        r = run_case(torch.tensor(f, device="cuda"), g, args.kind, 3, 0, args.alpha)
        rows.append(r)
        print(json.dumps(r), file=sys.stderr, flush=True)
    print(json.dumps({"kind": args.kind, "alpha": args.alpha, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
