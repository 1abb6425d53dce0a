"""Spread of the oracle's free-running 20-V-cycle energy under rounding-level perturbations.

The 64x64 configuration (sigma 0.05, alpha 20, J = 6, FP64 state, 20 V-cycles) is run once from
u_0 = f and then TRIALS times from u_0 = f (1 + 1e-15 z), z ~ N(0, 1) per pixel: a change of the
state at the level that a different summation order leaves after one sweep.  The energy is a
nonconvex function of a chaotic trajectory (the local arg-min sits on kinks of |kappa|), so the
trials end at slightly different energies.  The GPU computes every sum in another order; its
20-cycle energy is one more draw from the same spread.  Written to free_run_spread.json beside
this script; the GPU tests read their free-running energy tolerance from it.

    python tests/golden/free_run_spread.py [--trials 200] [--procs 8]

Calls only the oracle and the seeded input generator.
"""
import argparse
import json
import os
import sys
from concurrent.futures import ProcessPoolExecutor

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CASES = [  # (name, image seed, kind, fine colours)
    ("mean_4_seed0", 0, 0, 4),
    ("mean_4_seed1", 1, 0, 4),
    ("mean_4_seed2", 2, 0, 4),
    ("gauss_4_seed0", 0, 1, 4),
    ("mean_9_seed0", 0, 0, 9),
    ("gauss_9_seed0", 0, 1, 9),
]
H = W = 64
SIGMA, ALPHA, LEVELS, CYCLES = 0.05, 20.0, 6, 20


def _run(args):
    seed, kind, colours, trial = args
    import oracle
    from synth import noisy_image
    f, _ = noisy_image(H, W, seed, SIGMA)
    o = oracle.Oracle(H, W, ALPHA, kind, levels=LEVELS, fine_colours=colours, threads=1)
    u = f.copy()
    if trial >= 0:
        z = np.random.default_rng(10_000 * seed + 100 * kind + colours + 7919 * (trial + 1)).standard_normal(f.shape)
        u = f * (1.0 + 1e-15 * z)
    _, trace = o.solve(u, f, rel_tol=0.0, max_vcycles=CYCLES)
    return float(trace[-1])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trials", type=int, default=200)
    ap.add_argument("--procs", type=int, default=8)
    a = ap.parse_args()
    import oracle
    oracle.build(force=False)
    out = {"configuration": f"{H}x{W}, sigma {SIGMA}, alpha {ALPHA}, J {LEVELS}, FP64 state, {CYCLES} V-cycles",
           "perturbation": "u_0 = f (1 + 1e-15 z), z ~ N(0, 1) per pixel", "trials": a.trials, "cases": {}}
    with ProcessPoolExecutor(max_workers=a.procs) as ex:
        for name, seed, kind, colours in CASES:
            jobs = [(seed, kind, colours, t) for t in range(-1, a.trials)]
            es = list(ex.map(_run, jobs))
            ref, trials = es[0], np.array(es[1:])
            rel = np.sort(np.abs(trials - ref) / ref)
            out["cases"][name] = {
                "seed": seed, "kind": kind, "fine_colours": colours, "energy": ref,
                "rel_spread": {"median": float(np.median(rel)), "q90": float(np.quantile(rel, 0.9)),
                               "q99": float(np.quantile(rel, 0.99)), "max": float(rel[-1])},
                "energy_range": [float(trials.min()), float(trials.max())],
            }
            print(name, json.dumps(out["cases"][name]), flush=True)
    with open(os.path.join(HERE, "free_run_spread.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    main()
