"""Benchmark: Mpixel x V-cycles per second and time-to-energy-tolerance at 1024x1024.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

One step is one fine-to-coarse V-cycle of Algorithm 3 over a 1024x1024
synthetic image (all 10 levels, every colour sweep) followed by the FP64
energy reduction the stopping rule reads, exactly as the solver's loop runs it.
The image is resident on the GPU before timing starts.  After the timed steps
the script also runs full solves from u = f to a relative energy change below
1e-6 (mean and Gaussian curvature, noise sigma 0.1 and 0.05) and reports their wall time.

The roofline entry is for the dominant kernel (the pixel-level sweep): its
average launch time comes from HIP events around the pixel level on the
library's stream; its work is the algorithmic count of FP64 operations per
solved pixel (9 ring pixels x 51 local-energy evaluations x 40 flops for mean
curvature, 30 for Gaussian), with the count of the formulas the kernel
actually executes and the counter figures beside it.  The error of the
headline path against FP64 is stated from one V-cycle from u = f compared
with the C oracle's (float-state option and pure FP64).  The CPU baseline
times that oracle, built -O3 -march=native on this machine, on all the cores
the process may use (one V-cycle at 1024x1024) and on one core (one V-cycle of
a 512x512 image of the same family).  The large-image leg times 4096x4096 and
8192x8192 per level.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

H = W = 1024
ALPHA = 20.0
SIGMA = 0.1
SEED = 0

# FP64 operations (FMA = 2, add / multiply = 1; the hardware square-root estimate is not
# counted, its refinement is) that the pixel-level kernel executes per solved interior pixel,
# counted from its formulas.  The centre and the four diagonal ring pixels have a constant q, so
# their curvature is a polynomial in c with the constant factor folded in; each of the four edge
# neighbours evaluates N(c) (or D(c)) and q(c) from its moving first derivative w = w0 + s c and
# a refined 1/sqrt(q) (8 flops):
#   mean:     |K| evaluation 5 x 3 + 4 x 22 = 103,  derivative 5 x 4 + 4 x 32 = 148
#   Gaussian: |K| evaluation 5 x 5 + 4 x 18 = 97,   derivative 5 x 9 + 4 x 24 = 141
# Evaluations per pixel with M = 16 samples and G = 32 bisection steps: K(0), K(f*), 16 further
# samples and K at the bisection point (19), and 32 derivatives.
FLOPS_VALUE = {0: 103, 1: 97}
FLOPS_DERIV = {0: 148, 1: 141}
N_VALUE, N_DERIV = 19, 32
# The algorithmic work per solved pixel: 9 ring pixels, 51 local-energy evaluations (K(0), K(f*),
# 16 further samples, the bisection point and 32 derivatives), about 40 (mean) or 30 (Gaussian)
# FP64 flops per ring-pixel evaluation with the curvature's derivatives affine in c.
FLOPS_GENERAL_PIXEL = {0: 9 * 51 * 40, 1: 9 * 51 * 30}
FP64_PEAK_TFLOPS = 78.6   # MI355X vector FP64
HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
# Algorithmic HBM bytes per pixel and level in the float state: below block side 32 the colours
# interleave inside cache lines, so each of the 4 colour sweeps reads u and f and writes u
# (12 B/px); from side 32 on one pass over u and f and one write of u per level (12 B/px).
BYTES_PER_PX_LEVEL_FINE, BYTES_PER_PX_LEVEL_COARSE = 48, 12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--kind", type=int, default=0, help="0 mean curvature, 1 Gaussian curvature")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-solve", action="store_true", help="skip the time-to-tolerance solves")
    ap.add_argument("--cpu-vcycles", type=int, default=1)
    ap.add_argument("--no-large", action="store_true", help="skip the 4096^2 and 8192^2 per-level leg")
    ap.add_argument("--large-only", action="store_true",
                    help="run only the 4096^2 / 8192^2 leg and print its JSON (for profiling its kernels)")
    ap.add_argument("--large-sizes", default="4096,8192,1024x8192",
                    help="sides (N) or rows x columns (HxW); 1024x8192 is one GPU's row slab of 8192x8192 over 8 GPUs")
    ap.add_argument("--study", choices=["cycle", "fbs"],
                    help="run one study instead of the benchmark and print its JSON: 'cycle' = J x cycle shape x "
                         "block schedule of the exact path at 1024x1024, 'fbs' = the same for the paper's FBS step "
                         "and its image-size scaling (the size scaling of the exact path is --large-only "
                         "--large-sizes 1024,2048,4096,8192)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 256-image batched measurement")
    ap.add_argument("--batch-steps", type=int, default=3)
    ap.add_argument("--batch-solve", action="store_true", help="also solve all 256 images to 1e-6")
    ap.add_argument("--no-warm", action="store_true", help="skip the CNN warm-start comparison")
    ap.add_argument("--no-fbs", action="store_true", help="skip the paper's own local step (FBS) measurement")
    ap.add_argument("--no-recon", action="store_true", help="skip the reconstruction (b = A u + noise) measurement")
    ap.add_argument("--no-schedule", action="store_true",
                    help="skip the paper's 2^j - 1 block schedule measurement")
    ap.add_argument("--recon-only", action="store_true",
                    help="run only the reconstruction measurement and print its JSON (for profiling its kernels)")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 256-image batched measurement and print its JSON (for profiling its kernels)")
    ap.add_argument("--fbs-only", action="store_true",
                    help="run only the FBS measurement and print its JSON (for profiling its kernels)")
    ap.add_argument("--fbs-size", type=int, default=1024,
                    help="image side of --fbs-only; other than 1024 only the V-cycle rate is measured")
    ap.add_argument("--warm-batch", type=int, default=64,
                    help="also compare plain and warm-started batched solves on this many 1024x1024 images")
    return ap.parse_args()


# the sources the colour-sweep kernels are compiled from (their counters are void once these change)
SWEEP_SOURCES = ("mgc_device.h", "mgc_internal.h", "mgc_sweep.h", "mgc_kernels.hip", "mgc_split.hip")


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for name in SWEEP_SOURCES:
        with open(os.path.join(ROOT, "paper_2204_07921_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str, kernel_prefix: str):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    passes (already scaled by the copy-kernel calibration), or None when the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        doc = json.load(fh).get(workload_key)
    if not doc or doc.get("sources_sha") != kernel_sources_sha():
        return None
    for name, k in doc["kernels"].items():
        if name.startswith(kernel_prefix):
            return int(round((k["fetch_kib"] + k["write_kib"]) * 1024))
    return None


def warm_start_measure(fd, plain: dict, warm_batch: int) -> dict:
    """Time-to-energy-tol at 1024x1024 with the learned warm start: CNN forward (u0 = f + g(f)),
    then V-cycles until F <= F_plain (1 + 1e-6); if the budget (3x the plain V-cycles) runs out,
    the plain solve from u0 = f is run as the fallback and its time is added."""
    import torch
    from paper_2204_07921_amd import mgcurv, warmstart
    if not os.path.exists(warmstart.DEFAULT_WEIGHTS):
        return {"skipped": "no trained weights"}
    params, meta = warmstart.load()
    net = mgcurv.WarmStartCNN(H * W, params)
    solver = mgcurv.Solver(H, W, alpha=ALPHA, kind=0, dtype=torch.float32)
    target = plain["final_energy"] * (1 + 1e-6)
    f3 = fd.view(1, H, W)
    u0 = torch.empty_like(f3)
    net.forward(f3, u0)   # warm-up
    torch.cuda.synchronize()
    t = time.perf_counter()
    net.forward(f3, u0)
    res = solver.solve_target(u0.view(H, W), fd, target, max_vcycles=3 * plain["vcycles"] + 1)
    torch.cuda.synchronize()
    t_warm = time.perf_counter() - t
    fallback = res["status"] != 0
    if fallback:
        uu = fd.clone()
        t = time.perf_counter()
        solver.solve(uu, fd, rel_tol=1e-6, max_vcycles=2000)
        torch.cuda.synchronize()
        t_warm += time.perf_counter() - t
    out = {"weights": os.path.relpath(warmstart.DEFAULT_WEIGHTS, ROOT), "trained_on": {k: meta.get(k) for k in ("pairs", "size", "steps", "batch", "alpha", "kind")},
           "plain_seconds": plain["seconds"], "plain_vcycles": plain["vcycles"], "plain_energy": plain["final_energy"],
           "warm_seconds": round(t_warm, 4), "warm_vcycles": res["vcycles"], "warm_energy": res["energy"],
           "fallback": fallback, "energy_gap_rel": (res["energy"] - plain["final_energy"]) / plain["final_energy"],
           "speedup": round(plain["seconds"] / t_warm, 3)}
    # the same image with the nine-colour pixel level as the plain solver (it settles far lower; the
    # network's prediction starts above its energy and is refined)
    nine = warmstart.evaluate_single(net, fd.view(1, H, W), fine_colours=9)
    row = nine["per_image"][0]
    out["nine_colours"] = {"plain_seconds": round(row["plain_seconds"], 4), "plain_vcycles": row["plain_vcycles"],
                           "plain_energy": row["plain_energy"], "cnn_energy": row["cnn_energy"],
                           "warm_seconds": round(row["warm_seconds"], 4), "warm_vcycles": row["warm_vcycles"],
                           "warm_energy": row["warm_energy"], "fallback": row["fallback"],
                           "energy_gap_rel": (row["warm_energy"] - row["plain_energy"]) / row["plain_energy"],
                           "speedup": round(row["plain_seconds"] / row["warm_seconds"], 3)}
    if warm_batch:
        fe = warmstart.make_inputs(warm_batch, H, seed0=100000)
        net8 = mgcurv.WarmStartCNN(8 * H * W, params)
        out["cnn_inference"] = cnn_inference_measure(net8, fe)
        out["batch"] = warmstart.evaluate(net8, fe)
        # the nine-colour pixel level as the plain solver: it settles far lower, the network's
        # prediction starts above its energy, and the warm start has to refine
        nine = warmstart.evaluate_single(net8, fe, fine_colours=9)
        nine.pop("per_image")
        out["batch_nine_colours"] = nine
    return out


# Warm-start CNN inference per pixel: 4 hidden 32 -> 32 layers of 9 x 32 x 32 multiply-adds on the
# matrix cores, the 1 -> 32 and 32 -> 1 layers (9 x 32 each) on the vector units.  Bytes per pixel
# with the layers unfused (bfloat16 activations, 32 channels = 64 B): input layer 4 B in + 64 B
# out, each hidden layer 64 B in + 64 B out, output layer 64 B + 4 B (f) in + 4 B out.
CNN_MFMA_FLOPS_PX = 4 * 2 * 9 * 32 * 32
CNN_VALU_FLOPS_PX = 2 * 2 * 9 * 32
CNN_BYTES_PX = (4 + 64) + 4 * (64 + 64) + (64 + 4 + 4)
BF16_MFMA_PEAK_TFLOPS = 2500.0


def cnn_inference_measure(net, f) -> dict:
    """u0 = f + g(f) for a stack of 1024x1024 images in chunks of the network's capacity, HIP events on
    the current stream; rates against the bfloat16 matrix-core peak and the HBM peak."""
    import torch
    from paper_2204_07921_amd import warmstart
    warmstart.forward_chunked(net, f[:1].contiguous())
    stream = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    warmstart.forward_chunked(net, f)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    px = f.numel()
    return {"images": int(f.shape[0]), "ms": round(ms, 3), "ms_per_image": round(ms / f.shape[0], 4),
            "mfma_tflops": round(px * CNN_MFMA_FLOPS_PX / (ms * 1e-3) / 1e12, 2),
            "mfma_frac": round(px * CNN_MFMA_FLOPS_PX / (ms * 1e-3) / 1e12 / BF16_MFMA_PEAK_TFLOPS, 4),
            "algorithmic_gbs": round(px * CNN_BYTES_PX / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(px * CNN_BYTES_PX / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "counted_as": "matrix-core flops of the four 32->32 layers (2 x 9 x 32 x 32 per pixel each); "
                          "bytes of unfused bfloat16 layers (652 B per pixel)"}


def batch_measure(steps: int, solve: bool) -> dict:
    """256 images of sizes drawn from {128..1024}^2 (independent H, W), sigma ~ U[0.03, 0.12],
    alpha in {10, 20, 40}, mixed curvature kinds, float32 state: autotune, then time graph-replayed
    V-cycles (each with the per-image FP64 energies and their copy to the host)."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import batch_specs, noisy_image
    specs = batch_specs(256, seed=0)
    fs = [noisy_image(sp["height"], sp["width"], sp["seed"], sp["sigma"], dtype=np.float32)[0] for sp in specs]
    bs = mgcurv.BatchSolver(specs)
    fd = bs.pack(fs)
    mpx = bs.total / 1e6
    ud = fd.clone()
    t = time.perf_counter()
    bs.tune(ud, fd, repeats=1)
    torch.cuda.synchronize()
    tune_s = time.perf_counter() - t
    bs.solve(ud, fd, rel_tol=0.0, max_vcycles=1)  # warm-up: graph capture and first replay
    torch.cuda.synchronize()
    t = time.perf_counter()
    bs.solve(ud, fd, rel_tol=0.0, max_vcycles=steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t
    # algorithmic FP64 work of one V-cycle of the batch: per image, level by level, ring pixels per image
    # pixel (9 at b = 1, 8 / b above) x 51 evaluations x 40 (mean) or 30 (Gaussian) flops per ring pixel
    flops = 0.0
    for sp in specs:
        levels = max(1, int(np.ceil(np.log2(max(sp["height"], sp["width"])))))
        ring_per_px = 9.0 + sum(8.0 / (1 << (j - 1)) for j in range(2, levels + 1))
        flops += sp["height"] * sp["width"] * ring_per_px * 51 * (40 if sp["kind"] == 0 else 30)
    tflops = flops * steps / dt / 1e12
    out = {"workload": f"256 mixed images, {mpx:.1f} Mpixel, mean and Gaussian curvature, alpha 10/20/40",
           "value": round(mpx * steps / dt, 3), "unit": "Mpixel*V-cycles/s", "ms_per_vcycle": round(dt / steps * 1e3, 3),
           "algorithmic_tflops": round(tflops, 2), "fp64_frac": round(tflops / FP64_PEAK_TFLOPS, 4),
           "tune_seconds": round(tune_s, 2),
           "tuned": {str(l): bs.config(l) for l in range(1, bs.levels + 1)}}
    if solve:
        u2 = fd.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = bs.solve(u2, fd, rel_tol=1e-6, max_vcycles=400)
        torch.cuda.synchronize()
        out["solve_to_1e-6"] = {"seconds": round(time.perf_counter() - t, 3),
                                "vcycles_max": max(res["vcycles"]), "vcycles_mean": float(np.mean(res["vcycles"])),
                                "converged": int(sum(1 for x in res["image_status"] if x == 0))}
    bs.close()
    return out


def fbs_measure(steps: int, warmup: int, n: int = H) -> dict:
    """The paper's own local step (one FBS update per patch with tangent-plane estimates, patches
    of side 2^j - 1, J = 3) in the paper's intensity regime: the same kind of synthetic image
    scaled to [0, 255] with noise sigma 0.08 * 255, alpha 0.05.  Graph-replayed V-cycles per second
    at 1024 x 1024, then solves to relErr(u) < 1e-4 (the paper's rule) for both curvatures, with
    the energy and the RMSE to the clean image next to those of the exact local minimisation."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image
    f32, g = noisy_image(n, n, SEED, 0.08, dtype=np.float32)
    f32 = (255.0 * f32).astype(np.float32)
    g = 255.0 * g.astype(np.float64)
    fd = torch.tensor(f32, device="cuda")
    rmse = lambda u: float(np.sqrt(np.mean((u.detach().cpu().numpy().astype(np.float64) - g) ** 2)))
    out = {"workload": f"{n}x{n} synthetic image scaled to [0, 255], noise sigma 0.08 * 255, alpha 0.05, "
                       "J = 3 (patch sides 1, 3, 7), one FBS step per patch, float32 state, FP64 updates",
           "noise_rmse": round(rmse(fd), 4)}
    for kind, name in ((0, "mean"), (1, "gaussian")):
        s = mgcurv.FbsSolver(n, n, alpha=0.05, kind=kind, levels=3, dtype=torch.float32)
        u = fd.clone()
        for _ in range(warmup):
            s.vcycle(u, fd)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(steps):
            s.vcycle(u, fd)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t) / steps
        if n != H:
            out[name] = {"value": round(n * n / dt / 1e6, 3), "unit": "Mpixel*V-cycles/s",
                         "ms_per_vcycle": round(dt * 1e3, 4)}
            s.close()
            continue
        u = fd.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = s.solve(u, fd, tol=1e-4, max_vcycles=500, stop=mgcurv.MG_STOP_RELERR_U)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        ex = mgcurv.Solver(H, W, alpha=0.05, kind=kind, dtype=torch.float32)
        ue = fd.clone()
        rex = ex.solve(ue, fd, rel_tol=1e-6, max_vcycles=300)
        out[name] = {"value": round(n * n / dt / 1e6, 3), "unit": "Mpixel*V-cycles/s", "ms_per_vcycle": round(dt * 1e3, 4),
                     "solve_relerr_1e-4": {"seconds": round(el, 4), "vcycles": res["vcycles"], "status": res["status"],
                                           "energy": res["energy"], "rmse": round(rmse(u), 4)},
                     "exact_local_minimisation_1e-6": {"vcycles": rex["vcycles"], "energy": rex["energy"],
                                                       "rmse": round(rmse(ue), 4)}}
        s.close()
        ex.close()
    return out


def recon_measure(steps: int, warmup: int) -> dict:
    """Reconstruction from b = A g + noise (Section 5) at 1024 x 1024: A a 5 x 5 Gaussian blur
    (sigma 1, zero boundary), noise sigma 0.02 on the [0, 1] synthetic image, alpha 0.05, J = 3,
    20 CG iterations per colour, float32 state.  Graph-replayed V-cycles per second, then a solve
    to relErr(u) < 1e-4 with the RMSE to the clean image next to that of b."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image
    g, _ = noisy_image(H, W, SEED, 0.0, dtype=np.float64)
    # b = A g + noise, A applied by the library's own definition on the host (plain 5 x 5 sum)
    wts = np.exp(-np.add.outer(np.arange(-2, 3) ** 2, np.arange(-2, 3) ** 2) / 2.0)
    wts /= wts.sum()
    pad = np.zeros((H + 4, W + 4))
    pad[2:-2, 2:-2] = g
    ag = sum(wts[dy + 2, dx + 2] * pad[2 + dy:2 + dy + H, 2 + dx:2 + dx + W] for dy in range(-2, 3) for dx in range(-2, 3))
    b = (ag + 0.02 * np.random.default_rng(SEED + 1).standard_normal((H, W))).astype(np.float32)
    bd = torch.tensor(b, device="cuda")
    rmse = lambda u: float(np.sqrt(np.mean((u.detach().cpu().numpy().astype(np.float64) - g) ** 2)))
    s = mgcurv.ReconSolver(H, W, alpha=0.05, blur_sigma=1.0, levels=3, dtype=torch.float32, cg_iters=20)
    u = bd.clone()
    for _ in range(warmup):
        s.vcycle(u, bd)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        s.vcycle(u, bd)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t) / steps
    u = bd.clone()
    torch.cuda.synchronize()
    t = time.perf_counter()
    res = s.solve(u, bd, tol=1e-4, max_vcycles=200)
    torch.cuda.synchronize()
    el = time.perf_counter() - t
    out = {"workload": "1024x1024 synthetic image blurred by a 5x5 Gaussian (sigma 1) + noise 0.02, alpha 0.05, "
                       "J = 3, 20 CG iterations per colour, float32 state, FP64 CG",
           "value": round(H * W / dt / 1e6, 3), "unit": "Mpixel*V-cycles/s", "ms_per_vcycle": round(dt * 1e3, 4),
           "solve_relerr_1e-4": {"seconds": round(el, 4), "vcycles": res["vcycles"], "status": res["status"],
                                 "energy": res["energy"]},
           "rmse_b": round(rmse(bd), 5), "rmse_u": round(rmse(u), 5)}
    s.close()
    return out


def schedule_measure(fd, stream, kind: int, steps: int, warmup: int) -> dict:
    """The same image on the paper's block schedule (side 2^j - 1, Section 2.2) next to the nested
    power-of-two one: V-cycle rate, and solves from u = f to relErr(u) < 1e-4 (the rule of the
    paper's Tables 2-3)."""
    import torch
    from paper_2204_07921_amd import mgcurv
    out = {}
    for sched, name in ((1, "paper_2^j-1"), (0, "nested_2^(j-1)")):
        s = mgcurv.Solver(H, W, alpha=ALPHA, kind=kind, dtype=torch.float32, stream=stream, block_schedule=sched)
        u = fd.clone()
        for _ in range(warmup):
            s.vcycle(u, fd)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s.vcycle(u, fd)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        uu = fd.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = s.solve_rule(uu, fd, 1e-4, max_vcycles=400, stop=mgcurv.MG_STOP_RELERR_U)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        out[name] = {"levels": s.levels, "value": round(H * W / dt / 1e6, 3), "unit": "Mpixel*V-cycles/s",
                     "ms_per_vcycle": round(dt * 1e3, 4),
                     "relerr_1e-4": {"seconds": round(el, 4), "vcycles": res["vcycles"], "energy": res["energy"],
                                     "status": res["status"]}}
        s.close()
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_threads() -> int:
    """Threads the oracle may use: the process's CPU share (OMP_NUM_THREADS where the machine sets it),
    capped by the CPUs the process is allowed to run on."""
    try:
        avail = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        avail = os.cpu_count() or 1
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(avail, int(env))) if env.isdigit() else avail


def native_oracle():
    """The C oracle built -O3 -march=native for this machine into a temporary directory and selected
    for this process (FP64, no fast-math, no FMA contraction: the same values as the portable build)."""
    import tempfile
    import oracle
    from oracle import oracle as orc_mod
    path = os.path.join(tempfile.mkdtemp(prefix="mgc_oracle_"), "liboracle_native.so")
    oracle.build(force=True, out=path, native=True)
    os.environ["MGC_ORACLE_LIB"] = path
    orc_mod._lib = None
    return oracle


def cpu_baseline(f64: np.ndarray, kind: int, vcycles: int, u_gpu: np.ndarray, e_gpu: float,
                 u_gpu64: np.ndarray) -> tuple[dict, dict]:
    """The oracle timed on this machine's cores (float-state option, the GPU's state precision) and
    on one core (a 512x512 image of the same family); and the error of the GPU's first V-cycle
    from u = f against the float-state and the pure FP64 oracle."""
    from synth import noisy_image
    oracle = native_oracle()
    threads = cpu_threads()
    o = oracle.Oracle(H, W, ALPHA, kind, round_f32=True, threads=threads)
    u = f64.copy()
    t0 = time.perf_counter()
    for _ in range(vcycles):
        o.vcycle(u, f64)
    dt = time.perf_counter() - t0
    u_f32 = u
    if vcycles != 1:
        u_f32 = f64.copy()
        o.vcycle(u_f32, f64)
    o64 = oracle.Oracle(H, W, ALPHA, kind, threads=threads)
    u64 = f64.copy()
    t1 = time.perf_counter()
    o64.vcycle(u64, f64)
    dt64 = time.perf_counter() - t1
    e64 = o64.energy(u64, f64)
    h1 = w1 = 512
    f1 = noisy_image(h1, w1, SEED, SIGMA, dtype=np.float32)[0].astype(np.float64)
    o1 = oracle.Oracle(h1, w1, ALPHA, kind, round_f32=True, threads=1)
    u1 = f1.copy()
    t2 = time.perf_counter()
    o1.vcycle(u1, f1)
    dt1 = time.perf_counter() - t2
    base = {"value": round(H * W * vcycles / dt / 1e6, 4), "unit": "Mpixel*V-cycles/s", "cores": threads,
            "kind": "oracle",
            "sample": f"{vcycles} V-cycle(s) of the 1024x1024 image from u = f, FP64 C oracle (float-state option), "
                      f"-O3 -march=native, OpenMP over the blocks of a colour on {threads} threads, {dt:.1f} s",
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(h1 * w1 / dt1 / 1e6, 4), "unit": "Mpixel*V-cycles/s", "cores": 1,
                              "sample": f"1 V-cycle of a 512x512 image of the same family, {dt1:.1f} s"},
            "fp64_state_oracle": {"value": round(H * W / dt64 / 1e6, 4), "unit": "Mpixel*V-cycles/s",
                                  "cores": threads, "sample": f"1 V-cycle of the 1024x1024 image, {dt64:.1f} s"}}
    err = {"reference": "one V-cycle from u = f on the same float32 image; the C oracle in FP64 with its state "
                        "rounded to float after every update (float-state) and in pure FP64",
           "max_abs_u_vs_float_state_oracle": float(np.max(np.abs(u_gpu - u_f32))),
           "max_abs_u_vs_fp64_oracle": float(np.max(np.abs(u_gpu - u64))),
           "energy_rel_vs_fp64_oracle": abs(e_gpu - e64) / e64,
           "fp64_state_gpu_max_abs_u_vs_fp64_oracle": float(np.max(np.abs(u_gpu64 - u64)))}
    return base, err


def parse_sizes(text: str):
    """'4096,8192,1024x8192' -> [(4096, 4096), (8192, 8192), (1024, 8192)] (rows x columns)."""
    out = []
    for tok in text.split(","):
        tok = tok.strip().lower()
        if not tok:
            continue
        if "x" in tok:
            h, w = tok.split("x")
            out.append((int(h), int(w)))
        else:
            out.append((int(tok), int(tok)))
    return out


def large_measure(sizes, stream) -> dict:
    """4096x4096 (J = 12) and 8192x8192 (J = 13), sigma 0.1, float state, mean and Gaussian curvature:
    V-cycles per second and each level's time (HIP events on the library's stream), with the
    algorithmic HBM rate of each level against the 8 TB/s peak.  A rows x columns entry such as
    1024x8192 is one GPU's row slab of the 8192x8192 image split over 8 GPUs: its levels with
    blocks inside the slab are compared with the full image's same levels divided by 8."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image
    out = {}
    for hn, wn in sizes:
        f32, _ = noisy_image(hn, wn, SEED, SIGMA, dtype=np.float32)
        fd = torch.tensor(f32, device="cuda")
        del f32
        for kind in (0, 1):
            s = mgcurv.Solver(hn, wn, alpha=ALPHA, kind=kind, dtype=torch.float32, stream=stream)
            u = fd.clone()
            s.vcycle(u, fd)
            torch.cuda.synchronize()
            reps = 2
            t = time.perf_counter()
            for _ in range(reps):
                s.vcycle(u, fd)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            level_ms, level_gbs = [], []
            for level in range(1, s.levels + 1):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                s.level(u, fd, level)
                b.record(stream)
                torch.cuda.synchronize()
                ms = a.elapsed_time(b)
                side = 1 << (level - 1)
                bpp = BYTES_PER_PX_LEVEL_FINE if side < 32 else BYTES_PER_PX_LEVEL_COARSE
                level_ms.append(round(ms, 4))
                level_gbs.append(round(bpp * hn * wn / (ms * 1e-3) / 1e9, 1))
            e = s.energy(u, fd)
            out[f"{hn}x{wn}_{'mean' if kind == 0 else 'gaussian'}"] = {
                "levels": s.levels, "value": round(hn * wn / dt / 1e6, 3), "unit": "Mpixel*V-cycles/s",
                "ms_per_vcycle": round(dt * 1e3, 3), "level_ms": level_ms,
                "level_algorithmic_gbs": level_gbs,
                "level_hbm_frac": [round(g / HBM_PEAK_GBS, 4) for g in level_gbs],
                "energy_after_4_vcycles": e}
            s.close()
            del u
        del fd
        torch.cuda.empty_cache()
    # row slabs: the levels whose blocks stay inside the slab (side <= half its height) against the
    # full image's same levels over the number of slabs
    for (hn, wn) in sizes:
        full = (wn, wn)
        if hn >= wn or full not in sizes or wn % hn:
            continue
        parts = wn // hn
        local = max(1, (hn // 2).bit_length())   # levels 1 .. log2(hn / 2) + 1
        for kind in ("mean", "gaussian"):
            slab, whole = out[f"{hn}x{wn}_{kind}"], out[f"{wn}x{wn}_{kind}"]
            t_slab = sum(slab["level_ms"][:local])
            t_share = sum(whole["level_ms"][:local]) / parts
            out[f"{hn}x{wn}_{kind}"]["slab_of"] = {
                "image": f"{wn}x{wn}", "gpus": parts, "local_levels": local,
                "slab_ms_local_levels": round(t_slab, 4), "full_image_ms_same_levels_per_gpu": round(t_share, 4),
                "share_efficiency": round(t_share / t_slab, 3)}
    return out


def study_cycle(kind: int, tol: float = 1e-4, max_vcycles: int = 400) -> dict:
    """Level count, cycle shape and block schedule of the exact path (the experiments behind the
    paper's Tables 2-3, on the exact local minimisation): the 1024x1024 image (sigma 0.1, alpha 20,
    float state) solved from u = f to relErr(u) < tol with J = 1..10, half and full V-cycles, nested
    2^(j-1) blocks and the paper's 2^j - 1 patches; V-cycles, GPU time, energy, RMSE to the clean image."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image
    f32, g = noisy_image(H, W, SEED, SIGMA, dtype=np.float32)
    fd = torch.tensor(f32, device="cuda")
    rows = []
    for sched in (0, 1):
        for cycle in (0, 1):
            for J in range(1, 11):
                s = mgcurv.Solver(H, W, alpha=ALPHA, kind=kind, levels=J, dtype=torch.float32, cycle=cycle,
                                  block_schedule=sched)
                u = fd.clone()
                s.vcycle(u, fd)   # warm-up
                u = fd.clone()
                torch.cuda.synchronize()
                t = time.perf_counter()
                res = s.solve_rule(u, fd, tol, max_vcycles=max_vcycles, stop=mgcurv.MG_STOP_RELERR_U)
                torch.cuda.synchronize()
                el = time.perf_counter() - t
                rmse = float(np.sqrt(np.mean((u.cpu().numpy().astype(np.float64) - g) ** 2)))
                s.close()
                r = {"schedule": "2^j-1" if sched else "2^(j-1)", "levels": J, "cycle": "full" if cycle else "half",
                     "vcycles": res["vcycles"], "converged": res["status"] == 0, "seconds": round(el, 4),
                     "ms_per_vcycle": round(el / max(1, res["vcycles"]) * 1e3, 4), "energy": res["energy"],
                     "rmse": round(rmse, 5)}
                rows.append(r)
                print(json.dumps(r), file=sys.stderr, flush=True)
    return {"size": H, "kind": kind, "tol": tol, "rows": rows}


def study_fbs(kind: int, alpha: float = 0.05, sizes=(256, 512, 1024, 2048, 4096)) -> dict:
    """Level count, cycle shape and image size of the paper's own local step (one FBS update per
    patch, patches of side 2^j - 1) in the paper's intensity regime (the synthetic family scaled to
    [0, 255], noise 0.08 * 255): solves to relErr(u) < 1e-4 with J = 1..6, half and full V-cycles
    at 1024x1024, and J = 3 at the given sides."""
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image

    def image(n):
        f, g = noisy_image(n, n, 7, 0.08, dtype=np.float32)
        return torch.tensor((255.0 * f).astype(np.float32), device="cuda"), 255.0 * g.astype(np.float64)

    def run(fd, g, levels, cycle):
        n = fd.shape[0]
        s = mgcurv.FbsSolver(n, n, alpha=alpha, kind=kind, levels=levels, dtype=torch.float32, cycle=cycle)
        u = fd.clone()
        s.solve(u, fd, tol=1e-4, max_vcycles=1, stop=mgcurv.MG_STOP_RELERR_U)   # capture and warm up
        u = fd.clone()
        torch.cuda.synchronize()
        t = time.perf_counter()
        res = s.solve(u, fd, tol=1e-4, max_vcycles=500, stop=mgcurv.MG_STOP_RELERR_U)
        torch.cuda.synchronize()
        el = time.perf_counter() - t
        rmse = float(np.sqrt(np.mean((u.cpu().numpy().astype(np.float64) - g) ** 2)))
        s.close()
        r = {"size": n, "levels": levels, "cycle": "full" if cycle else "half", "vcycles": res["vcycles"],
             "converged": res["status"] == 0, "seconds": round(el, 5),
             "ms_per_vcycle": round(el / max(1, res["vcycles"]) * 1e3, 4), "energy": res["energy"],
             "rmse": round(rmse, 4)}
        print(json.dumps(r), file=sys.stderr, flush=True)
        return r

    rows = []
    fd, g = image(1024)
    for cycle in (0, 1):
        for J in range(1, 7):
            rows.append(run(fd, g, J, cycle))
    for n in sizes:
        fd, g = image(n)
        rows.append(run(fd, g, 3, 0))
    return {"kind": kind, "alpha": alpha, "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only (the path has no multi-GPU "
                          "sharding)", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.fbs_only:
        print(json.dumps({"fbs": fbs_measure(args.steps, args.warmup, args.fbs_size)}), flush=True)
        return
    if args.recon_only:
        print(json.dumps({"recon": recon_measure(args.steps, args.warmup)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batch": batch_measure(args.batch_steps, args.batch_solve)}), flush=True)
        return
    if args.study:
        fn = {"cycle": lambda: study_cycle(args.kind), "fbs": lambda: study_fbs(args.kind)}[args.study]
        print(json.dumps({"study_" + args.study: fn()}), flush=True)
        return
    if args.large_only:
        import torch
        print(json.dumps({"large": large_measure(parse_sizes(args.large_sizes), torch.cuda.current_stream())}),
              flush=True)
        return
    import torch
    from paper_2204_07921_amd import mgcurv
    from synth import noisy_image

    f32, _ = noisy_image(H, W, SEED, SIGMA, dtype=np.float32)
    f64 = f32.astype(np.float64)
    dev = torch.device("cuda:0")
    fd = torch.tensor(f32, device=dev)
    stream = torch.cuda.current_stream()
    solver = mgcurv.Solver(H, W, alpha=ALPHA, kind=args.kind, dtype=torch.float32, stream=stream)
    J = solver.levels

    # --- timed V-cycles -------------------------------------------------------------
    u = fd.clone()
    for _ in range(args.warmup):
        solver.vcycle(u, fd, want_energy=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    energies = []
    for _ in range(args.steps):
        energies.append(solver.vcycle(u, fd, want_energy=True))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt / args.steps * 1e3
    value = H * W * args.steps / dt / 1e6

    # --- dominant kernel: pixel-level sweep, HIP events on the library's stream -----
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    reps = 5
    ev0.record(stream)
    for _ in range(reps):
        solver.level(u, fd, 1)
    ev1.record(stream)
    torch.cuda.synchronize()
    launches = reps * 4
    avg_ms = ev0.elapsed_time(ev1) / launches
    pixels_per_launch = (H // 2) * (W // 2)
    flops_executed = pixels_per_launch * (N_VALUE * FLOPS_VALUE[args.kind] + N_DERIV * FLOPS_DERIV[args.kind])
    flops_launch = pixels_per_launch * FLOPS_GENERAL_PIXEL[args.kind]
    achieved = flops_launch / (avg_ms * 1e-3) / 1e12

    # --- error against FP64: one V-cycle from u = f (float state), and the FP64-state mode ---
    u1 = fd.clone()
    e1 = solver.vcycle(u1, fd, want_energy=True)
    u1_host = u1.cpu().numpy().astype(np.float64)
    f64d = torch.tensor(f64, device=dev)
    s64 = mgcurv.Solver(H, W, alpha=ALPHA, kind=args.kind, dtype=torch.float64, stream=stream)
    u64d = f64d.clone()
    s64.vcycle(u64d, f64d)
    u1_64_host = u64d.cpu().numpy()
    for _ in range(args.warmup):
        s64.vcycle(u64d, f64d)
    torch.cuda.synchronize()
    t64 = time.perf_counter()
    for _ in range(args.steps):
        s64.vcycle(u64d, f64d, want_energy=True)
    torch.cuda.synchronize()
    dt64 = time.perf_counter() - t64
    fp64_state = {"value": round(H * W * args.steps / dt64 / 1e6, 3), "unit": "Mpixel*V-cycles/s",
                  "ms_per_step": round(dt64 / args.steps * 1e3, 4),
                  "note": "the same step with the state u, f held in float64"}
    s64.close()
    del u64d, f64d

    # per-level times (one V-cycle's share), for the report
    level_ms = []
    for level in range(1, J + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        solver.level(u, fd, level)
        b.record(stream)
        torch.cuda.synchronize()
        level_ms.append(round(a.elapsed_time(b), 4))

    # --- time to energy tolerance ---------------------------------------------------
    solves = {}
    if not args.no_solve:
        f05 = torch.tensor(noisy_image(H, W, SEED, 0.05, dtype=np.float32)[0], device=dev)
        # (sigma, image, kind, pixel-level colours): the four-colour runs of both curvatures, and the
        # mean-curvature runs with the nine-colour pixel level, which settles far lower
        runs = [(sg, im, k, 4) for sg, im in ((SIGMA, fd), (0.05, f05)) for k in (0, 1)]
        runs += [(SIGMA, fd, 0, 9), (0.05, f05, 0, 9)]
        for sigma, fs, kind, colours in runs:
            s = mgcurv.Solver(H, W, alpha=ALPHA, kind=kind, dtype=torch.float32, stream=stream,
                              fine_colours=colours)
            uu = fs.clone()
            torch.cuda.synchronize()
            t = time.perf_counter()
            # at sigma 0.05 the mean-curvature energy creeps down by ~1.45e-6 of itself per
            # V-cycle, above the 1e-6 rule, so that solve is capped and reports the last change
            res = s.solve(uu, fs, rel_tol=1e-6, max_vcycles=2000 if sigma == SIGMA else 400, trace=True)
            torch.cuda.synchronize()
            el = time.perf_counter() - t
            tr = res["trace"]
            name = (("mean" if kind == 0 else "gaussian") + ("" if sigma == SIGMA else "_sigma_0.05")
                    + ("" if colours == 4 else "_9_colours"))
            solves[name] = {"seconds": round(el, 4), "vcycles": res["vcycles"], "final_energy": res["energy"],
                            "status": res["status"],
                            "last_rel_change": abs(tr[-1] - tr[-2]) / abs(tr[-1]) if len(tr) > 1 else None}
            s.close()

    out = {
        "metric": "Mpixel*V-cycles/s (1024x1024, plain multigrid; time-to-energy-tol in solves)",
        "value": round(value, 3),
        "unit": "Mpixel*V-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "dtype_note": "every local minimisation and the energy compute in FP64; the state u, f is stored as float32",
        "data": "synthetic",
        "config": {"workload": "1024x1024 piecewise-smooth image + Gaussian noise sigma 0.1, "
                               f"{'mean' if args.kind == 0 else 'Gaussian'} curvature, alpha 20, {J} levels, "
                               "4 colours, float32 state, FP64 local minimisation and energy",
                   "image": [H, W], "levels": J, "alpha": ALPHA, "sigma": SIGMA,
                   "state_dtype": "f32", "local_math": "f64", "samples": 16, "bisections": 32},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": round(achieved / FP64_PEAK_TFLOPS, 4),
                     "traffic": measured_traffic(f"1024x1024_{'mean' if args.kind == 0 else 'gauss'}_f32",
                                                 f"mgc::sweep_pixels_kernel<float, {args.kind}"),
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "kernel": "sweep_pixels_kernel (b = 1)", "avg_launch_ms": round(avg_ms, 5),
                     "flops_per_launch": flops_launch,
                     "flops_counted_as": "algorithmic: per solved pixel 9 ring pixels x 51 local-energy "
                                         "evaluations x 40 (mean) or 30 (Gaussian) FP64 flops",
                     "executed_formula_tflops": round(flops_executed / (avg_ms * 1e-3) / 1e12, 3),
                     "executed_formula_flops_per_launch": flops_executed,
                     "note": "one launch = one colour of the pixel level (outer ring of cells on 16-lane "
                             "groups, interior cells one thread each), timed with HIP events on the library stream"},
        "level_ms": level_ms,
        "fp64_state": fp64_state,
        "energy_last": energies[-1],
        "time_to_tol": solves,
    }
    if not args.no_schedule:
        out["block_schedule"] = schedule_measure(fd, stream, args.kind, args.steps, args.warmup)
    if not args.no_warm and "mean" in solves:
        out["warm_start"] = warm_start_measure(fd, solves["mean"], args.warm_batch)
    if not args.no_batch:
        out["batch"] = batch_measure(args.batch_steps, args.batch_solve)
    if not args.no_fbs:
        out["fbs"] = fbs_measure(max(args.steps, 20), args.warmup)
    if not args.no_recon:
        out["recon"] = recon_measure(5, 1)
    if not args.no_large:
        out["large"] = large_measure(parse_sizes(args.large_sizes), stream)
    if not args.no_cpu:
        out["cpu_baseline"], out["error_vs_fp64"] = cpu_baseline(f64, args.kind, args.cpu_vcycles, u1_host, e1,
                                                                 u1_64_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
