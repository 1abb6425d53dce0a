"""Size study of the exact path (the large-scale configurations): for square synthetic images of
side 1024 .. 8192 (sigma 0.1, alpha 20, J = log2 of the side, float32 state) it reports the
V-cycle time, Mpixel*V-cycles/s, and per level the time of the level's four colour sweeps with
the HBM rate they would need if they moved only their algorithmic bytes.

Algorithmic bytes of a level (float32 state): on levels b >= 2 every pixel is read from u and f
and written once over the four colours, 12 B per pixel; on the pixel level each of the four
launches reads u over the whole image, f at its colour's pixels and writes the whole other
buffer (two-phase update), 9 B per pixel per launch, 36 B per pixel per level.

    python -m paper_2204_07921_amd.scale_study [--sizes 1024 2048 4096 8192] [--kind 0]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np
import torch

from . import mgcurv


def _time(fn, reps: int) -> float:
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def run_size(n: int, kind: int, reps: int) -> dict:
    from synth import noisy_image
    f32, _ = noisy_image(n, n, 0, 0.1, dtype=np.float32)
    fd = torch.tensor(f32, device="cuda")
    s = mgcurv.Solver(n, n, alpha=20.0, kind=kind, dtype=torch.float32, stream=torch.cuda.current_stream())
    u = fd.clone()
    s.vcycle(u, fd)
    vc = _time(lambda: s.vcycle(u, fd), reps)
    levels = []
    for level in range(1, s.levels + 1):
        ms = _time(lambda: s.level(u, fd, level), reps)
        px = n * n
        bytes_level = (36 if level == 1 else 12) * px
        levels.append({"level": level, "b": 1 << (level - 1), "ms": round(ms, 4),
                       "algorithmic_GBps": round(bytes_level / (ms * 1e-3) / 1e9, 1)})
    s.close()
    return {"size": n, "kind": kind, "levels_J": len(levels), "vcycle_ms": round(vc, 4),
            "mpx_vcycles_per_s": round(n * n / (vc * 1e-3) / 1e6, 1), "per_level": levels}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", type=int, nargs="+", default=[1024, 2048, 4096, 8192])
    ap.add_argument("--kind", type=int, nargs="+", default=[0, 1])
    ap.add_argument("--reps", type=int, default=5)
    args = ap.parse_args()
    rows = []
    for kind in args.kind:
        for n in args.sizes:
            r = run_size(n, kind, args.reps)
            rows.append(r)
            print(json.dumps({k: v for k, v in r.items() if k != "per_level"}), file=sys.stderr, flush=True)
    print(json.dumps({"rows": rows}), flush=True)


if __name__ == "__main__":
    main()
