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


@pytest.mark.parametrize("kind", [0, 1])
def test_counted_flops_per_pixel(kind):
    """The executed-formula count per solved pixel: 19 value and 32 derivative evaluations."""
    per_pixel = bench.N_VALUE * bench.FLOPS_VALUE[kind] + bench.N_DERIV * bench.FLOPS_DERIV[kind]
    assert per_pixel == {0: 6693, 1: 6355}[kind]
    assert bench.N_VALUE + bench.N_DERIV == 2 + 16 + 1 + 32
