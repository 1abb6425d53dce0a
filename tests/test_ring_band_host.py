"""The block-ring enumeration of the colour-sweep kernels (`ring_band` / `band_at`, host and
device code) against brute force on the CPU: built with hipcc for the host and run here."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_ring_band_covers_every_ring_pixel(tmp_path):
    exe = str(tmp_path / "ring_band_check")
    subprocess.check_call([_hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-Wno-unused-command-line-argument",
                           os.path.join(HERE, "host", "ring_band_check.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "bad 0" in r.stdout


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_ring_band_check_is_clean_under_sanitizers(tmp_path):
    """The same host check built with the address and undefined-behaviour sanitizers (host code only;
    nothing runs on a GPU)."""
    exe = str(tmp_path / "ring_band_check_san")
    subprocess.check_call([_hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                           "-Wno-unused-command-line-argument",
                           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-sanitize-recover=all",
                           os.path.join(HERE, "host", "ring_band_check.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    sys.stdout.write(r.stdout + r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "bad 0" in r.stdout


def test_oracle_is_clean_under_sanitizers(tmp_path):
    """The C oracle built with the address and undefined-behaviour sanitizers and driven through
    solves, every local solve of every level, sweeps and the FBS path on ragged images down to
    2 x 2, all options, one and four threads (tests/host/oracle_sanitize.c)."""
    root = os.path.dirname(HERE)
    exe = str(tmp_path / "oracle_san")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-ffp-contract=off",
                           os.path.join(HERE, "host", "oracle_sanitize.c"),
                           os.path.join(root, "oracle", "mgc_oracle.c"), os.path.join(root, "oracle", "fbs_oracle.c"),
                           "-o", exe, "-lm"])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    sys.stdout.write(r.stdout + r.stderr[-2000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized runs" in r.stdout


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_split_tree_and_depth_host_check(tmp_path):
    """The split coarse solve's bisection tree against sequential bisection (bitwise, d = 1..8,
    G = 0..64, monotone and arbitrary signs) and its depth choice against its constraints."""
    exe = str(tmp_path / "split_tree_check")
    subprocess.check_call([_hipcc(), "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                           "-Wno-unused-command-line-argument",
                           os.path.join(HERE, "host", "split_tree_check.cpp"), "-o", exe],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    sys.stdout.write(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "bad 0" in r.stdout
