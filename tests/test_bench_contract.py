"""CPU checks of bench.py's host-side contract: it refuses more than one GPU before touching a
device, and the roofline's `traffic` comes from the committed counter summary only while the
kernel sources are the ones the counters were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_follows_the_kernel_sources(monkeypatch):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    doc = json.load(open(path))
    entry = doc["1024x1024_mean_f32"]
    k = next(v for n, v in entry["kernels"].items() if n.startswith("mgc::sweep_pixels_kernel<float, 0"))
    expect = int(round((k["fetch_kib"] + k["write_kib"]) * 1024))
    # sources equal to those the counters saw: fetch + write bytes of the kernel
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: entry["sources_sha"])
    assert bench.measured_traffic("1024x1024_mean_f32", "mgc::sweep_pixels_kernel<float, 0") == expect
    # an unknown workload or kernel gives no figure
    assert bench.measured_traffic("no_such_workload", "mgc::") is None
    assert bench.measured_traffic("1024x1024_mean_f32", "no_such_kernel") is None
    # once the sources differ from those the counters saw, the figure is withdrawn
    monkeypatch.setattr(bench, "kernel_sources_sha", lambda: "0" * 16)
    assert bench.measured_traffic("1024x1024_mean_f32", "mgc::sweep_pixels_kernel<float, 0") is None


_VCYCLE_DIGEST = """
import hashlib, sys
import numpy as np
sys.path.insert(0, {root!r})
import oracle
from synth import noisy_image
f, _ = noisy_image(40, 48, 3, 0.1)
out = []
for kind in (0, 1):
    o = oracle.Oracle(40, 48, 20.0, kind, threads=2)
    u = f.copy()
    o.solve(u, f, rel_tol=0.0, max_vcycles=2)
    out.append(hashlib.sha256(u.tobytes()).hexdigest())
print(" ".join(out))
"""


def _digest(env_lib):
    env = dict(os.environ)
    env.pop("MGC_ORACLE_LIB", None)
    if env_lib:
        env["MGC_ORACLE_LIB"] = env_lib
    r = subprocess.run([sys.executable, "-c", _VCYCLE_DIGEST.format(root=ROOT)], env=env, capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    return r.stdout.strip()


def test_native_oracle_build_gives_the_same_values(tmp_path):
    """The CPU baseline times the oracle built -O3 -march=native; without fast-math and with FMA
    contraction off its results are those of the portable build bit for bit."""
    import oracle
    native = oracle.build(force=True, out=str(tmp_path / "liboracle_native.so"), native=True)
    assert _digest(native) == _digest(None)


def test_cpu_threads_follow_the_process_share(monkeypatch):
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert bench.cpu_threads() == min(3, len(os.sched_getaffinity(0)))
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert bench.cpu_threads() == len(os.sched_getaffinity(0))


def test_large_sizes_parse_squares_and_slabs():
    import bench
    assert bench.parse_sizes("4096, 8192,1024x8192") == [(4096, 4096), (8192, 8192), (1024, 8192)]
    assert bench.parse_sizes("") == []
