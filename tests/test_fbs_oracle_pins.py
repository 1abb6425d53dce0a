"""Pins of the FBS oracle (the paper's own local step) against what the paper and the
mathematics fix, independently of the oracle's code:

* eq. (distance to tri) as printed, for the four axis planes of the finest level;
* a plane fitted through the three surface points by a linear solve (not the oracle's cross
  product) for every plane of every ring, border patches included, with the ring's
  planes enumerated here from their definition (lines through the centre, third vertices
  perpendicular to them) rather than from the oracle's table;
* eq. (c-sol2) as the minimiser of eq. (quadratic) found by a scalar minimiser, and the
  step-size schedule of Algorithm 2;
* Proposition 2's selection by brute force, a cylinder's vanishing Gaussian estimate and
  Proposition 1's flattening of a bowl;
* the patch grid of Section 2.2 (m_j = ceil(m / (2^j - 1)), 2^(j+2) planes), the colour
  map and the non-interaction of patches of one colour (order-independence);
* fixed points, invariances and the alpha limit.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.optimize import minimize_scalar

from oracle import FbsOracle
from oracle.oracle import curvature_map

MC, GC = 0, 1


def _rand(h, w, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal((h, w))


# --- independent geometry -------------------------------------------------------------

def _ring_planes(r):
    """The 8 planes of ring r from their definition: each line through the centre joins
    two opposite ring pixels; its third vertices are the ring pixels perpendicular to it.
    Returned in the order W-E, N-S, NW-SE, NE-SW, each with its two thirds ordered by
    the row offset, then the column offset (N before S, W before E, NE before SW,
    NW before SE)."""
    lines = [((0, -r), (0, r)), ((-r, 0), (r, 0)), ((-r, -r), (r, r)), ((-r, r), (r, -r))]
    ring = [(di * r, dj * r) for di in (-1, 0, 1) for dj in (-1, 0, 1) if (di, dj) != (0, 0)]
    out = []
    for a, b in lines:
        thirds = [t for t in ring if t[0] * (b[0] - a[0]) + t[1] * (b[1] - a[1]) == 0]
        assert len(thirds) == 2
        thirds.sort()
        out.extend((a, b, t) for t in thirds)
    return out


def _value(u, i, j, box, c):
    h, w = u.shape
    ci, cj = min(max(i, 0), h - 1), min(max(j, 0), w - 1)
    v = u[ci, cj]
    r0, r1, c0, c1 = box
    if r0 <= ci < r1 and c0 <= cj < c1:
        v += c
    return v


def _plane_fit(u, centre, box, c, a, b, t):
    """Signed distance (plane above the centre point > 0) by fitting z = k0 + k1 x + k2 y
    through the three points with a linear solve; ds2 = squared half chord a-b in 3-D."""
    oi, oj = centre
    pts = [(di, dj, _value(u, oi + di, oj + dj, box, c)) for di, dj in (a, b, t)]
    A = np.array([[1.0, p[0], p[1]] for p in pts])
    k = np.linalg.solve(A, np.array([p[2] for p in pts]))
    zo = _value(u, oi, oj, box, c)
    d = (k[0] - zo) / math.sqrt(1.0 + k[1] ** 2 + k[2] ** 2)
    ds2 = 0.25 * sum((pts[1][m] - pts[0][m]) ** 2 for m in range(3))
    return d, ds2


def _centre_and_box(o, level, p, q):
    b = o.block_side(level)
    r0, r1, c0, c1 = o.block_bounds(level, p, q)
    return (r0 + (b - 1) // 2, c0 + (b - 1) // 2), (r0, r1, c0, c1)


# --- pins -----------------------------------------------------------------------------

def test_distance_matches_printed_formula():
    """eq. (distance to tri): d = (u_W + u_E - 2u_C) / sqrt((u_W + u_E - 2u_N)^2 + (u_E - u_W)^2 + 4)
    for the plane through the row neighbours and the pixel above; the other axis planes are
    the same formula on the reflected / transposed neighbourhood."""
    rng = np.random.default_rng(1)
    for trial in range(50):
        u = rng.standard_normal((5, 5)) * (0.2 + trial / 10)
        o = FbsOracle(5, 5, 1.0)
        C, N, S, W, E = u[2, 2], u[1, 2], u[3, 2], u[2, 1], u[2, 3]

        def printed(ul, ur, uo, uc):
            return (ul + ur - 2 * uc) / math.sqrt((ul + ur - 2 * uo) ** 2 + (ur - ul) ** 2 + 4)

        expect = [printed(W, E, N, C), printed(W, E, S, C), printed(N, S, W, C), printed(N, S, E, C)]
        for k in range(4):
            d, _ = o.plane(u, 1, 2, 2, 1, k)
            assert d == pytest.approx(expect[k], rel=1e-13, abs=1e-15), (trial, k)


@pytest.mark.parametrize("level", [1, 2, 3])
@pytest.mark.parametrize("shape", [(23, 19), (9, 30)])
def test_every_plane_against_a_plane_fit(level, shape):
    h, w = shape
    o = FbsOracle(h, w, 1.0, levels=level)
    u = _rand(h, w, 7 + level)
    mj, nj = o.grid(level)
    for p, q in itertools.product(range(mj), range(nj)):
        centre, box = _centre_and_box(o, level, p, q)
        c = 0.37 * ((p + 2 * q) % 3 - 1)
        for r in range(1, o.rings(level) + 1):
            for k, (a, b, t) in enumerate(_ring_planes(r)):
                d_ref, ds2_ref = _plane_fit(u, centre, box, c, a, b, t)
                d, ds2 = o.plane(u, level, p, q, r, k, c)
                assert d == pytest.approx(d_ref, rel=1e-10, abs=1e-12), (p, q, r, k)
                assert ds2 == pytest.approx(ds2_ref, rel=1e-12), (p, q, r, k)


def test_plane_count_per_level():
    """Section 2.2: iota = 2^(j+2) tangent planes on level j (8 on the finest)."""
    o = FbsOracle(8, 8, 1.0)
    for j in range(1, 8):
        assert o.L.fbs_planes(j) == 2 ** (j + 2)
        assert 8 * o.rings(j) == 2 ** (j + 2)


def test_affine_surface_has_zero_distances_and_is_fixed():
    """Three points of a plane span that plane, so every distance vanishes where the taps
    stay inside the image (the replicated prolongation bends an affine surface at the
    border); a constant image is a fixed point of the whole V-cycle."""
    h, w = 17, 21
    ii, jj = np.mgrid[0:h, 0:w]
    f = (3 * ii - 2 * jj + 5).astype(np.float64)
    for kind in (MC, GC):
        o = FbsOracle(h, w, 20.0, kind, levels=3, steps=2)
        checked = 0
        for level in (1, 2, 3):
            mj, nj = o.grid(level)
            R = o.rings(level)
            for p, q in itertools.product(range(mj), range(nj)):
                (oi, oj), _ = _centre_and_box(o, level, p, q)
                if not (R <= oi < h - R and R <= oj < w - R):
                    continue
                for r in range(1, R + 1):
                    for k in range(8):
                        assert o.plane(f, level, p, q, r, k)[0] == 0.0
                        checked += 1
        assert checked > 500
        g = np.full((h, w), 0.625)
        u = g.copy()
        for _ in range(3):
            o.vcycle(u, g)
        assert np.array_equal(u, g)


@pytest.mark.parametrize("kind", [MC, GC])
def test_backward_step_minimises_the_quadratic(kind):
    """eq. (c-sol2) / its patch form: c_{t+1} minimises
    alpha s/2 (c - f*)^2 + (c - c_t)^2 / (2 eta_t) + (c - c_{t+1/2})^2 / (2 eta_t);
    eta_0 = 1, eta_{t+1} = 1/sqrt(1 + t) (Algorithm 2)."""
    h, w = 20, 20
    u = _rand(h, w, 3, 0.3)
    f = u + _rand(h, w, 4, 0.1)
    for alpha in (0.0, 0.05, 3.0, 20.0):
        o = FbsOracle(h, w, alpha, kind, levels=3, steps=6)
        for level, (p, q) in [(1, (4, 5)), (2, (1, 2)), (3, (1, 1)), (3, (2, 2))]:
            c, tr, s, fs = o.block_step(u, f, level, p, q)
            assert np.allclose(tr[:, 2], [1.0] + [1.0 / math.sqrt(1 + t) for t in range(5)], rtol=0, atol=1e-15)
            for t in range(6):
                ct, half, eta = tr[t]
                nxt = tr[t + 1, 0] if t < 5 else c
                obj = lambda x: 0.5 * alpha * s * (x - fs) ** 2 + (x - ct) ** 2 / (2 * eta) + (x - half) ** 2 / (2 * eta)
                lo, hi = sorted([min(ct, half, fs) - 1.0, max(ct, half, fs) + 1.0])
                ref = minimize_scalar(obj, bounds=(lo, hi), method="bounded", options={"xatol": 1e-12}).x
                assert nxt == pytest.approx(ref, abs=1e-8), (alpha, level, t)


def test_patch_mean_and_size():
    h, w = 23, 17
    u = _rand(h, w, 5)
    f = _rand(h, w, 6)
    o = FbsOracle(h, w, 1.0, levels=4)
    for level in (1, 2, 3, 4):
        mj, nj = o.grid(level)
        assert (mj, nj) == (math.ceil(h / (2 ** level - 1)), math.ceil(w / (2 ** level - 1)))
        for p, q in itertools.product(range(mj), range(nj)):
            r0, r1, c0, c1 = o.block_bounds(level, p, q)
            _, _, s, fs = o.block_step(u, f, level, p, q)
            assert s == (r1 - r0) * (c1 - c0)
            assert fs == pytest.approx(np.mean(f[r0:r1, c0:c1] - u[r0:r1, c0:c1]), rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("level", [1, 2, 3])
def test_forward_estimates_brute_force(level):
    """Proposition 1: mean of all iota distances; Proposition 2: distance to the plane whose
    normal curvature d/ds^2 is the extreme (first min / first max) of smaller magnitude;
    both taken on the state with the patch shifted by c_t (so c_{t+1/2} - c_t is the
    estimate there)."""
    h, w = 19, 22
    u = _rand(h, w, 11, 0.5)
    f = u + _rand(h, w, 12, 0.1)
    for kind in (MC, GC):
        o = FbsOracle(h, w, 2.0, kind, levels=level, steps=3)
        mj, nj = o.grid(level)
        for p, q in itertools.product(range(mj), range(nj)):
            centre, box = _centre_and_box(o, level, p, q)
            c, tr, _, _ = o.block_step(u, f, level, p, q)
            for t in range(3):
                ct, half, _ = tr[t]
                ds = []
                for r in range(1, o.rings(level) + 1):
                    for a, b, tv in _ring_planes(r):
                        ds.append(_plane_fit(u, centre, box, ct, a, b, tv))
                d = np.array([x[0] for x in ds])
                kap = np.array([x[0] / x[1] for x in ds])
                if kind == MC:
                    est = d.mean()
                else:
                    imin, imax = int(np.argmin(kap)), int(np.argmax(kap))
                    est = d[imin] if abs(kap[imin]) <= abs(kap[imax]) else d[imax]
                assert half - ct == pytest.approx(est, rel=1e-9, abs=1e-12), (kind, p, q, t)


def test_gaussian_estimate_vanishes_on_a_cylinder():
    """u varying along the columns only: every plane containing the N-S line through the centre
    holds the centre point, so one principal curvature is 0 and Proposition 2 gives c = d* = 0."""
    h, w = 15, 15
    jj = np.mgrid[0:h, 0:w][1].astype(np.float64)
    u = 0.05 * (jj - 7.3) ** 2
    o = FbsOracle(h, w, 0.0, GC, levels=3)
    om = FbsOracle(h, w, 0.0, MC, levels=3)
    for level, (p, q) in [(1, (7, 7)), (2, (2, 2)), (3, (1, 1))]:
        assert o.estimate(u, level, p, q) == 0.0
        assert om.estimate(u, level, p, q) > 0.0


def test_mean_estimate_flattens_a_bowl():
    """Proposition 1: on a bowl the planes lie above the centre, and moving the centre by the
    estimate lowers its discrete mean curvature magnitude."""
    h, w = 9, 9
    ii, jj = np.mgrid[0:h, 0:w].astype(np.float64)
    for a, b in [(0.2, 0.2), (0.3, 0.1), (1.5, 0.7)]:
        u = 0.5 * (a * (ii - 4) ** 2 + b * (jj - 4) ** 2)
        o = FbsOracle(h, w, 0.0, MC, levels=1)
        d = o.estimate(u, 1, 4, 4)
        assert d > 0
        v = u.copy()
        v[4, 4] += d
        assert abs(curvature_map(MC, v)[4, 4]) < abs(curvature_map(MC, u)[4, 4])


@pytest.mark.parametrize("kind", [MC, GC])
def test_colour_sweep_is_order_independent(kind):
    """Patches of one colour do not interact (Section 2.3): applying their updates one at a
    time, in a shuffled order, gives the Jacobi sweep bit for bit."""
    h, w = 23, 19
    f = _rand(h, w, 21, 0.4)
    u0 = f + _rand(h, w, 22, 0.1)
    rng = np.random.default_rng(5)
    for level in (1, 2, 3):
        o = FbsOracle(h, w, 5.0, kind, levels=3, steps=2)
        for colour in range(4):
            ref = u0.copy()
            cgrid = o.sweep(ref, f, level, colour, want_c=True)
            seq = u0.copy()
            mj, nj = o.grid(level)
            blocks = [(p, q) for p in range(mj) for q in range(nj) if o.colour_of(p, q) == colour]
            rng.shuffle(blocks)
            for p, q in blocks:
                c, _, _, _ = o.block_step(seq, f, level, p, q)
                assert c == cgrid[p, q]
                r0, r1, c0, c1 = o.block_bounds(level, p, q)
                seq[r0:r1, c0:c1] += c
            assert np.array_equal(seq, ref), (level, colour)


def test_colour_map_and_neighbours():
    o = FbsOracle(40, 40, 1.0)
    for p in range(6):
        for q in range(6):
            assert o.colour_of(p, q) == 2 * (p % 2) + (q % 2)
            for dp, dq in itertools.product((-1, 0, 1), repeat=2):
                if (dp, dq) != (0, 0):
                    assert o.colour_of(p + 2 + dp, q + 2 + dq) != o.colour_of(p + 2, q + 2)


@pytest.mark.parametrize("kind", [MC, GC])
def test_transpose_symmetry_of_self_mapped_colours(kind):
    """Transposing u and f maps colour 0 and colour 3 onto themselves; their sweeps commute
    with the transpose (the plane set is closed under it)."""
    n = 21
    f = _rand(n, n, 31, 0.4)
    u0 = f + _rand(n, n, 32, 0.1)
    o = FbsOracle(n, n, 5.0, kind, levels=3, steps=2)
    for level in (1, 2, 3):
        for colour in (0, 3):
            a = u0.copy()
            o.sweep(a, f, level, colour)
            b = np.ascontiguousarray(u0.T)
            o.sweep(b, np.ascontiguousarray(f.T), level, colour)
            assert np.allclose(a, b.T, rtol=0, atol=1e-12), (level, colour)


@pytest.mark.parametrize("kind", [MC, GC])
def test_shift_and_negation(kind):
    h, w = 26, 31
    f = _rand(h, w, 41, 0.3)
    o = FbsOracle(h, w, 10.0, kind, levels=3, steps=1)
    base = f.copy()
    for _ in range(3):
        o.vcycle(base, f)
    sh = f + 2.5
    o_sh = sh.copy()
    for _ in range(3):
        o.vcycle(o_sh, sh)
    assert np.allclose(o_sh - 2.5, base, rtol=0, atol=1e-12)
    neg = -f
    u_neg = neg.copy()
    for _ in range(3):
        o.vcycle(u_neg, neg)
    assert np.array_equal(u_neg, -base)


def test_alpha_limit_restores_f():
    h, w = 16, 18
    f = _rand(h, w, 51, 0.3)
    u = f + _rand(h, w, 52, 0.2)
    o = FbsOracle(h, w, 1e12, MC, levels=1)
    o.level(u, f, 1)
    assert np.allclose(u, f, rtol=0, atol=1e-9)


def test_relerr_stop_rule():
    """Section 4: relErr(u) = ||u_l - u_{l-1}|| / ||u_l|| < tol ends the iteration."""
    h, w = 24, 24
    f = _rand(h, w, 61, 0.3) + 1.0
    o = FbsOracle(h, w, 20.0, MC, levels=3)
    u = f.copy()
    n, _ = o.solve(u, f, tol=1e-4, max_vcycles=200, stop=1)
    assert 1 <= n < 200
    # replay: the rule holds at step n and fails before it
    v = f.copy()
    for l in range(1, n + 1):
        prev = v.copy()
        o.vcycle(v, f)
        rel = np.linalg.norm(v - prev) / np.linalg.norm(v)
        assert (rel < 1e-4) == (l == n), l
    assert np.array_equal(u, v)
