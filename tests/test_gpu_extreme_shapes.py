"""Extreme shapes through the C ABI.

* Aspect ratios far from square (2 x 65536, 65536 x 3, 5 x 40000): J = 16 levels whose blocks are
  clipped to a few rows or columns; every colour sweep of a whole V-cycle against the oracle, pixel
  by pixel (FP64 state).
* The largest image the ABI accepts: 46340 x 46340 = 2,147,395,600 pixels (just under 2^31), float
  state (u, f and the pixel level's second buffer take 26 GB).  One whole V-cycle runs (all 16
  levels, blocks of side 1024 .. 32768 streaming their ring records); then the pixel level and the
  side-2048 level are swept once more and checked at the image's far corner, where every index and
  byte offset is largest, against the oracle's local solves on a crop of that corner (the crop
  keeps the true right and bottom borders and a 3-pixel margin inside the image on the other two
  sides, so the oracle's ring and taps equal those of the full image)."""
import numpy as np
import pytest
import torch

from synth import noisy_image
from tests.parity_helpers import full_grid_check

pytestmark = pytest.mark.gpu


def _case(msg):
    print(f"\n[case] {msg}", flush=True)


@pytest.mark.parametrize("shape", [(2, 65536), (65536, 3), (5, 40000)])
def test_extreme_aspect_ratio_every_sweep(orc, shape):
    from paper_2204_07921_amd import mgcurv as mg
    h, w = shape
    f, _ = noisy_image(h, w, 21, 0.1)
    s = mg.Solver(h, w, alpha=20.0, kind=0, dtype=torch.float64)
    o = orc.Oracle(h, w, 20.0, 0, threads=8)
    assert s.levels == o.levels == 16
    fd = torch.tensor(f, device="cuda")
    ug = fd.clone()
    equal = blocks = 0
    for level in range(1, s.levels + 1):
        for colour in range(4):
            _case(f"aspect {shape} level {level} colour {colour}")
            before = ug.cpu().numpy()
            s.sweep(ug, fd, level, colour)
            after = ug.cpu().numpy()
            nb, ne, _ = full_grid_check(o, f, before, after, level, colour, fp64=True)
            blocks += nb
            equal += ne
    print(f"{blocks} blocks, {equal} on the equal-minimum criterion")
    assert equal <= max(2, blocks // 1000)


def test_near_maximum_image_size(orc):
    from paper_2204_07921_amd import mgcurv as mg
    H = W = 46340
    assert H * W <= 2 ** 31 - 1
    _case(f"max size {H}x{W}: build the image")
    tile = torch.tensor(noisy_image(1024, 1024, 33, 0.1, dtype=np.float32)[0], device="cuda")
    reps = -(-H // 1024)
    fd = tile.repeat(reps, reps)[:H, :W].contiguous()
    del tile
    torch.cuda.empty_cache()
    s = mg.Solver(H, W, alpha=20.0, kind=0, dtype=torch.float32)
    assert s.levels == 16
    ug = fd.clone()
    _case("max size: one V-cycle")
    e = s.vcycle(ug, fd, want_energy=True)
    assert np.isfinite(e) and e > 0.0

    def crop(t, r0, c0):
        return t[r0:, c0:].cpu().numpy().astype(np.float64)

    # pixel level, colour 3, bottom-right 40 x 40 corner
    _case("max size: pixel level at the far corner")
    R0, C0 = H - 40, W - 40
    fc = crop(fd, R0, C0)
    before = crop(ug, R0, C0)
    s.sweep(ug, fd, 1, 3)
    after = crop(ug, R0, C0)
    oc = orc.Oracle(40, 40, 20.0, 0, round_f32=True)
    checked = 0
    for i in range(3, 40):
        for j in range(3, 40):
            gi, gj = R0 + i, C0 + j
            if 2 * (gi % 2) + (gj % 2) != 3:
                assert after[i, j] == before[i, j], (gi, gj)
                continue
            info = oc.local_solve(before, fc, (i, i + 1, j, j + 1))
            expect = np.float64(np.float32(before[i, j] + info.c))
            assert after[i, j] == expect, (gi, gj, after[i, j], expect)
            checked += 1
    assert checked >= 300
    # side 2048 (level 12, streamed ring records): the block at the far corner
    _case("max size: side-2048 level at the far corner")
    b = 2048
    p, q = (H - 1) // b, (W - 1) // b
    colour = 2 * (p % 2) + (q % 2)
    r0, c0 = p * b, q * b
    R0, C0 = r0 - 3, c0 - 3
    fc = crop(fd, R0, C0)
    before = crop(ug, R0, C0)
    s.sweep(ug, fd, 12, colour)
    after = crop(ug, R0, C0)
    hc, wc = before.shape
    oc = orc.Oracle(hc, wc, 20.0, 0, round_f32=True, threads=8)
    info = oc.local_solve(before, fc, (3, hc, 3, wc))
    expect = (before[3:, 3:] + info.c).astype(np.float32).astype(np.float64)
    print(f"corner block c = {info.c:.6e} (accepted {info.accepted})")
    assert np.array_equal(after[3:, 3:], expect)
    assert np.array_equal(after[:3, :], before[:3, :]) and np.array_equal(after[:, :3], before[:, :3])
