"""Level-count and cycle-shape study of the exact path (the experiments behind Tables 2-3 of
the paper, on the exact local minimisation): for a synthetic 1024 x 1024 image (sigma 0.1,
alpha 20, mean curvature, float32 state) it solves to relErr(u) < tol from u = f with J = 1 .. 10
levels, half and full V-cycles, nested power-of-two blocks and the paper's 2^j - 1 patches, and
reports V-cycles, GPU time, final energy and RMSE to the clean image.

    python -m paper_2204_07921_amd.cycle_study [--tol 1e-4] [--kind 0] [--size 1024] [--schedules 0 1]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import mgcurv


def main():
    from synth import noisy_image
    ap = argparse.ArgumentParser()
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--kind", type=int, default=0)
    ap.add_argument("--tol", type=float, default=1e-4)
    ap.add_argument("--max-vcycles", type=int, default=400)
    ap.add_argument("--levels", type=int, nargs="+", default=list(range(1, 11)))
    ap.add_argument("--schedules", type=int, nargs="+", default=[0, 1],
                    help="block sides 0: 2^(j-1), 1: 2^j - 1 (Section 2.2)")
    args = ap.parse_args()
    n = args.size
    f32, g = noisy_image(n, n, 0, 0.1, dtype=np.float32)
    fd = torch.tensor(f32, device="cuda")
    rows = []
    for sched, cycle, J in [(a, b, c) for a in args.schedules for b in (0, 1) for c in args.levels]:
        s = mgcurv.Solver(n, n, alpha=20.0, kind=args.kind, levels=J, dtype=torch.float32, cycle=cycle,
                          block_schedule=sched)
        u = fd.clone()
        s.vcycle(u, fd)   # warm-up
        u = fd.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = s.solve_rule(u, fd, args.tol, max_vcycles=args.max_vcycles, stop=mgcurv.MG_STOP_RELERR_U)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        rmse = float(np.sqrt(np.mean((u.cpu().numpy().astype(np.float64) - g) ** 2)))
        s.close()
        r = {"schedule": "2^j-1" if sched else "2^(j-1)", "levels": J, "cycle": "full" if cycle else "half",
             "vcycles": res["vcycles"],
             "converged": res["status"] == 0, "seconds": round(el, 4),
             "ms_per_vcycle": round(el / max(1, res["vcycles"]) * 1e3, 4), "energy": res["energy"],
             "rmse": round(rmse, 5)}
        rows.append(r)
        print(json.dumps(r), file=sys.stderr, flush=True)
    print(json.dumps({"size": n, "kind": args.kind, "tol": args.tol, "rows": rows}), flush=True)


if __name__ == "__main__":
    main()
