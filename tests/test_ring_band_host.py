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
