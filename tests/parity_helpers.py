"""Shared checks for the GPU parity tests (teacher-forced comparison of one colour sweep)."""
import numpy as np


def _blocks_of(o, level, colour):
    m, n = o.grid(level)
    return [(p, q) for p in range(m) for q in range(n) if o.colour_of(level, p, q) == colour]


def colour_mask(o, level, colour):
    """Boolean H x W mask of the pixels that belong to blocks of `colour` at `level` (block (p, q) of
    side b covers rows [pb, (p+1)b) and columns [qb, (q+1)b), clipped to the image)."""
    b = o.block_side(level)
    p = np.arange(o.p.height) // b
    q = np.arange(o.p.width) // b
    if o.num_colours(level) == 9:
        col = 3 * (p[:, None] % 3) + (q[None, :] % 3)
    else:
        col = 2 * (p[:, None] % 2) + (q[None, :] % 2)
    return col == colour


def assert_untouched(o, before, after, level, colour):
    """A colour sweep leaves every pixel outside the colour's blocks bitwise unchanged."""
    outside = ~colour_mask(o, level, colour)
    assert np.array_equal(after[outside], before[outside]), \
        (level, colour, int(np.count_nonzero(after[outside] != before[outside])))


def _check_sweep_against_oracle(o, f, before, after, level, colour, fp64=True):
    """Teacher-forced parity of one colour sweep: the oracle solves every block of the colour from the
    GPU's own input state.  A block passes if its correction matches to 1e-10 (FP64 state; in FP32 the
    rounded block values must match), or, where the arg-min is ill-conditioned (a minimum on a kink of
    |kappa| with a tiny slope), if the GPU's correction reaches the same local-energy minimum
    (oracle's Delta at the GPU's c within 1e-12 (1 + V0) of the oracle's own).  Returns
    (max |dc|, number of blocks that needed the equal-minimum criterion)."""
    assert_untouched(o, before, after, level, colour)
    worst, n_equal = 0.0, 0
    for p, q in _blocks_of(o, level, colour):
        bnd = o.block_bounds(level, p, q)
        r0, r1, c0, c1 = bnd
        info = o.local_solve(before, f, bnd)
        c_gpu = after[r0, c0] - before[r0, c0]
        if fp64:
            dc = abs(c_gpu - info.c)
            ok = dc <= 1e-10
        else:
            expect = (before[r0:r1, c0:c1] + info.c).astype(np.float32).astype(np.float64)
            dc = float(np.max(np.abs(after[r0:r1, c0:c1] - expect)))
            ok = dc == 0.0
        # every pixel of the block moved by the same c
        assert np.allclose(after[r0:r1, c0:c1] - before[r0:r1, c0:c1], c_gpu, rtol=0, atol=1e-6 if not fp64 else 1e-13)
        if not ok:
            v0 = info.K0 + 0.5 * o.p.alpha * info.s * info.fs ** 2
            d_gpu = o.local_delta(before, f, bnd, c_gpu)
            d_orc = o.local_delta(before, f, bnd, info.c)
            assert d_gpu <= d_orc + 1e-12 * (1 + v0) + (0 if fp64 else 1e-7 * (1 + v0)), \
                (level, colour, p, q, c_gpu, info.c, d_gpu, d_orc)
            n_equal += 1
        worst = max(worst, dc)
    return worst, n_equal


def full_grid_check(o, f, before, after, level, colour, fp64):
    """Full-grid teacher-forced parity of one colour sweep: the oracle sweeps the GPU's own input
    state, then every pixel is compared.  Pixels outside the colour stay bitwise unchanged; inside,
    a block passes if its pixels equal the oracle's (FP64 state: to 1e-10; float state: bitwise,
    both sides rounding the same FP64 correction to float), or, where the arg-min is ill-conditioned,
    if the GPU's correction reaches the same local-energy minimum (the oracle's Delta at the GPU's c
    within 1e-12 (1 + V0) of its own).  Returns (number of blocks of the colour, blocks that needed
    the equal-minimum criterion, max |u_gpu - u_oracle| over the other blocks)."""
    assert_untouched(o, before, after, level, colour)
    x = before.copy()
    o.sweep(x, f, level, colour)
    mask = colour_mask(o, level, colour)
    d = np.abs(after - x)
    bad = (d > 1e-10) if fp64 else (d != 0.0)
    b = o.block_side(level)
    rows, cols = np.nonzero(bad)
    bad_blocks = sorted(set(zip((rows // b).tolist(), (cols // b).tolist())))
    n_blocks = int(np.count_nonzero(mask[::b, ::b]))
    for p, q in bad_blocks:
        bnd = o.block_bounds(level, p, q)
        r0, r1, c0, c1 = bnd
        c_gpu = after[r0, c0] - before[r0, c0]
        # every pixel of the block moved by the same correction
        assert np.allclose(after[r0:r1, c0:c1] - before[r0:r1, c0:c1], c_gpu, rtol=0,
                           atol=1e-13 if fp64 else 1e-6)
        info = o.local_solve(before, f, bnd)
        v0 = info.K0 + 0.5 * o.p.alpha * info.s * info.fs ** 2
        d_gpu = o.local_delta(before, f, bnd, c_gpu)
        d_orc = o.local_delta(before, f, bnd, info.c)
        assert d_gpu <= d_orc + 1e-12 * (1 + v0) + (0 if fp64 else 1e-7 * (1 + v0)), \
            (level, colour, p, q, c_gpu, info.c, d_gpu, d_orc)
    good = np.ones_like(bad)
    for p, q in bad_blocks:
        r0, r1, c0, c1 = o.block_bounds(level, p, q)
        good[r0:r1, c0:c1] = False
    worst = float(d[good].max()) if good.any() else 0.0
    return n_blocks, len(bad_blocks), worst


def _check_batch_sweeps_against_oracle(mg, orc, bs, fs, ud, fd, levels, schedule=0, threads=8):
    """Every image of a batch against the float-state oracle, sweep by sweep from the batch's own state."""
    oracles = [orc.Oracle(sp["height"], sp["width"], sp["alpha"], sp["kind"], round_f32=True, threads=threads,
                          schedule=schedule) for sp in bs.specs]
    f64 = [f.astype(np.float64) for f in fs]
    for level in levels:
        if level == 1:
            # the pixel level runs all four colours in one call; check colour by colour through
            # the oracle's Jacobi semantics by composing its four sweeps
            before = [v.cpu().numpy().astype(np.float64) for v in bs.unpack(ud)]
            bs.level(ud, fd, 1)
            after = [v.cpu().numpy().astype(np.float64) for v in bs.unpack(ud)]
            for k, o in enumerate(oracles):
                if level > o.levels:
                    continue
                x = before[k].copy()
                for colour in range(4):
                    o.sweep(x, f64[k], 1, colour)
                # composed over four colours; an FP64 rounding tie may move one float by an ulp
                diff = np.abs(x - after[k])
                assert diff.max() <= 1e-5 and np.count_nonzero(diff) <= max(1, diff.size // 1000), k
            continue
        for colour in range(4):
            before = [v.cpu().numpy().astype(np.float64) for v in bs.unpack(ud)]
            bs.sweep(ud, fd, level, colour)
            after = [v.cpu().numpy().astype(np.float64) for v in bs.unpack(ud)]
            for k, o in enumerate(oracles):
                if level > o.levels:
                    assert np.array_equal(before[k], after[k])
                    continue
                _, n_equal = _check_sweep_against_oracle(o, f64[k], before[k], after[k], level, colour, fp64=False)
                assert n_equal <= 1, (k, level, colour)
