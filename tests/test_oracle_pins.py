"""Pins of the FP64 CPU oracle against facts that do not come from the oracle itself.

Each test names what it pins (see the oracle's header for the readings R1-R8):
closed-form curvatures of analytic surfaces, the ring identity against the
whole-image energy, the minimiser bracket, brute-force minimisation on tiny
images, monotonicity, fixed points, invariances, limits and colour
separability.
"""
import json
import math
import os

import numpy as np
import pytest

from synth import noisy_image

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "curvature_closed_forms.json")


def _surface(case, X, Y):
    s, p = case["surface"], case["params"]
    if s == "sphere":
        return np.sqrt(p["R"] ** 2 - X ** 2 - Y ** 2)
    if s == "cylinder":
        return np.sqrt(p["R"] ** 2 - X ** 2)
    if s == "helicoid":
        return np.arctan(Y / X)
    if s == "saddle":
        return X * Y
    if s == "scherk_rotated":
        a = p["angle"]
        Xr = np.cos(a) * X - np.sin(a) * Y
        Yr = np.sin(a) * X + np.cos(a) * Y
        return np.log(np.cos(Yr) / np.cos(Xr))
    if s == "paraboloid":
        return 0.5 * (p["a"] * X ** 2 + p["b"] * Y ** 2)
    raise KeyError(s)


def _fd_curvature(orc, kind, case, h):
    # 5x5 samples centred on (x, y); row index grows with y.
    off = (np.arange(5) - 2) * h
    X = case["x"] + off[None, :]
    Y = case["y"] + off[:, None]
    u = np.ascontiguousarray(_surface(case, X + 0 * Y, Y + 0 * X))
    return orc.oracle.curvature_map(kind, u, h)[2, 2]


@pytest.mark.parametrize("kind", [0, 1])
def test_p1_closed_form_curvatures(orc, kind):
    """P1: 3x3 central differences converge at second order to the closed forms."""
    doc = json.load(open(GOLDEN))
    key = "mc" if kind == 0 else "gc"
    for case in doc["cases"]:
        exact = case[key]
        if exact is None:
            continue
        e1 = abs(_fd_curvature(orc, kind, case, 1e-2) - exact)
        e2 = abs(_fd_curvature(orc, kind, case, 5e-3) - exact)
        scale = 1.0 + abs(exact)
        if case["surface"] in ("saddle", "paraboloid"):
            # quadratics: the stencils are exact
            assert e1 < 1e-12 * scale, (case["surface"], e1)
            continue
        if case["surface"] == "cylinder" and kind == 1:
            assert e1 == 0.0, e1  # u_yy = u_xy = 0 exactly
            continue
        assert e1 < 1e-3 * scale, (case["surface"], key, e1)
        assert e2 < e1, (case["surface"], key, e1, e2)
        order = math.log(e1 / e2, 2)
        assert 1.8 < order < 2.2, (case["surface"], key, order)


def test_p1_plane_and_flip(orc):
    """Planes have zero curvature away from the border; flipping y leaves both curvatures unchanged."""
    H, W = 12, 9
    i, j = np.mgrid[0:H, 0:W]
    plane = (i * 0.375 - j * 0.125).astype(np.float64)
    for kind in (0, 1):
        k = orc.oracle.curvature_map(kind, plane, 1.0)
        assert np.all(k[1:-1, 1:-1] == 0.0)
    f, _ = noisy_image(16, 20, 3, 0.1)
    for kind in (0, 1):
        k = orc.oracle.curvature_map(kind, f, 1.0)
        kf = orc.oracle.curvature_map(kind, np.ascontiguousarray(f[::-1]), 1.0)[::-1]
        kt = orc.oracle.curvature_map(kind, np.ascontiguousarray(f.T), 1.0).T
        assert np.allclose(k, kf, rtol=0, atol=1e-13)
        assert np.allclose(k, kt, rtol=0, atol=1e-13)


def _blocks(o, level):
    m, n = o.grid(level)
    for p in range(m):
        for q in range(n):
            yield p, q, o.block_bounds(level, p, q)


@pytest.mark.parametrize("kind", [0, 1])
def test_p2_ring_identity(orc, kind):
    """P2: Delta(c) on the ring equals F(u + c chi_B) - F(u) on the whole image (edges, corners, clipped blocks)."""
    H, W = 13, 11  # odd sizes give clipped blocks at every level
    f, _ = noisy_image(H, W, 5, 0.1)
    rng = np.random.default_rng(1)
    u = f + 0.05 * rng.standard_normal(f.shape)
    o = orc.Oracle(H, W, 20.0, kind)
    E0 = o.energy(u, f)
    for level in range(1, o.levels + 1):
        for p, q, (r0, r1, c0, c1) in _blocks(o, level):
            c = float(rng.uniform(-0.3, 0.3))
            v = u.copy()
            v[r0:r1, c0:c1] += c
            full = o.energy(v, f) - E0
            loc = o.local_delta(u, f, (r0, r1, c0, c1), c)
            assert abs(full - loc) < 1e-10 * (1 + abs(E0)), (level, p, q, full, loc)


def test_p2_ring_size(orc):
    """Ring sizes: 9 for an interior pixel, 8b for an interior block of side b >= 2."""
    H = W = 64
    u = np.zeros((H, W))
    o = orc.Oracle(H, W, 20.0, 0)
    assert o.ring_size(u, (30, 31, 30, 31)) == 9
    for b in (2, 4, 8, 16):
        r0 = 16
        assert o.ring_size(u, (r0, r0 + b, r0, r0 + b)) == 8 * b
    # the top-left corner pixel: only pixels of the 2x2 corner see it
    assert o.ring_size(u, (0, 1, 0, 1)) == 4


@pytest.mark.parametrize("kind", [0, 1])
def test_derivative_matches_finite_differences(orc, kind):
    """The ring derivative K'(c) agrees with central differences of K(c) away from kinks."""
    f, _ = noisy_image(16, 16, 7, 0.1)
    o = orc.Oracle(16, 16, 20.0, kind)
    rng = np.random.default_rng(2)
    checked = 0
    for level in (1, 2, 3):
        for p, q, bnd in list(_blocks(o, level))[:12]:
            for c in rng.uniform(-0.5, 0.5, size=6):
                h = 1e-6
                km, k0, kp = o.ring_K_many(f, bnd, [c - h, c, c + h])
                curv = abs(kp - 2 * k0 + km) / h ** 2
                if curv > 1e3:  # a kink of |kappa| inside [c - h, c + h]
                    continue
                fd = (kp - km) / (2 * h)
                d = o.ring_dK(f, bnd, c)
                assert abs(fd - d) < 1e-5 * (1 + abs(d)), (level, p, q, c, fd, d)
                checked += 1
    assert checked > 100


def _brute_min(o, u, bnd, fs, s, lo, hi, n=4001):
    """Dense grid + local refinement of V(c) on [lo, hi]; independent of the oracle's search."""
    a = o.p.alpha * s
    cs = np.linspace(lo, hi, n)
    v = o.ring_K_many(u, bnd, cs) + 0.5 * a * (cs - fs) ** 2
    k = int(np.argmin(v))
    best_c, best_v = cs[k], v[k]
    span = (hi - lo) / (n - 1)
    for _ in range(6):  # zoom in around the best grid point
        cs = np.linspace(best_c - span, best_c + span, 201)
        v = o.ring_K_many(u, bnd, cs) + 0.5 * a * (cs - fs) ** 2
        k = int(np.argmin(v))
        if v[k] <= best_v:
            best_c, best_v = cs[k], v[k]
        span = 2 * span / 200
    return best_c, best_v


@pytest.mark.parametrize("kind", [0, 1])
def test_p3_p4_local_solve_vs_brute_force(orc, kind):
    """P3: the global minimiser lies in [f* - rho, f* + rho].
    P4: the local solver reaches the brute-force minimum of the local energy on 8x8 images."""
    worst = 0.0
    n_blocks = 0
    for seed in range(12):
        f, _ = noisy_image(8, 8, 100 + seed, 0.1)
        rng = np.random.default_rng(seed)
        u = f + 0.08 * rng.standard_normal(f.shape)
        o = orc.Oracle(8, 8, 20.0, kind)
        for level in (1, 2, 3):
            for p, q, bnd in _blocks(o, level):
                info = o.local_solve(u, f, bnd)
                fs, s, rho = info.fs, info.s, info.rho
                a = 20.0 * s
                # P3: a wide search (3 rho on each side) finds its minimum inside the bracket
                wide = max(rho, 1e-3)
                c_bf, v_bf = _brute_min(o, u, bnd, fs, s, fs - 3 * wide, fs + 3 * wide, n=3001)
                assert abs(c_bf - fs) <= rho + 2e-3 * wide, (seed, level, p, q, c_bf, fs, rho)
                # P4: the algorithm's choice is as good as the brute-force minimum
                def V(c):
                    return o.ring_K(u, bnd, c) + 0.5 * a * (c - fs) ** 2
                v_alg = V(info.c_tilde)
                K0 = info.K0
                gap = v_alg - v_bf
                worst = max(worst, gap / (1 + K0))
                assert gap <= 1e-9 * (1 + K0), (seed, level, p, q, v_alg, v_bf, info.c_tilde, c_bf)
                # accept rule: a returned correction lowers the local energy by more than eta
                eta = 1e-12 * (1 + K0 + 0.5 * a * fs * fs)
                assert (info.accepted and info.delta < -eta) or (not info.accepted and info.c == 0.0)
                if info.accepted:
                    assert info.c == info.c_tilde
                n_blocks += 1
    assert n_blocks == 12 * (64 + 16 + 4)


@pytest.mark.parametrize("kind", [0, 1])
def test_p5_p9_monotone_and_separable(orc, kind):
    """P5 + P9: for b >= 2 (and for b = 1 with nine colours) one colour sweep changes F by exactly
    the sum of the blocks' local changes, each <= 0, so F never increases."""
    H, W = 24, 20
    f, _ = noisy_image(H, W, 11, 0.08)
    for colours in (4, 9):
        o = orc.Oracle(H, W, 20.0, kind, fine_colours=colours)
        u = f.copy()
        for cycle in range(2):
            for level in range(1, o.levels + 1):
                if level == 1 and colours == 4:
                    # Jacobi within a colour at b = 1: same-colour pixels share ring pixels
                    for colour in range(4):
                        o.sweep(u, f, level, colour)
                    continue
                for colour in range(o.num_colours(level)):
                    E0 = o.energy(u, f)
                    deltas = []
                    for p, q, bnd in _blocks(o, level):
                        if o.colour_of(level, p, q) != colour:
                            continue
                        info = o.local_solve(u, f, bnd)
                        deltas.append(info.delta if info.accepted else 0.0)
                    o.sweep(u, f, level, colour)
                    E1 = o.energy(u, f)
                    # accept rule: every applied block lowers its local energy
                    assert all(d <= 0.0 for d in deltas)
                    assert abs((E1 - E0) - sum(deltas)) < 1e-10 * (1 + E0), (level, colour, E1 - E0, sum(deltas))
                    assert E1 <= E0 + 1e-10 * (1 + E0)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("colours", [4, 9])
def test_pixel_level_sweep_is_jacobi_within_colour(orc, kind, colours):
    """Reading R7 at b = 1: every pixel of a colour takes the local solver's correction computed from
    the state at the start of the colour, and all of them are added afterwards (with four colours,
    same-colour pixels two apart share ring pixels, so applying them one by one would change later
    corrections).  The expected state is assembled here pixel by pixel from single-block solves on
    the frozen start state; the sweep must equal it bitwise, and every other pixel stays untouched.
    The colour pattern is written here, not taken from the oracle."""
    H, W = 22, 19
    f, _ = noisy_image(H, W, 31, 0.1)
    o = orc.Oracle(H, W, 20.0, kind, fine_colours=colours)
    u = f.copy()
    o.vcycle(u, f)   # a state away from u = f, where many pixels move
    moved, changed_neighbour = 0, 0
    for colour in range(colours):
        before = u.copy()
        expect = u.copy()
        for i in range(H):
            for j in range(W):
                own = 3 * (i % 3) + (j % 3) if colours == 9 else 2 * (i % 2) + (j % 2)
                if own != colour:
                    continue
                c = o.local_solve(before, f, (i, i + 1, j, j + 1)).c
                expect[i, j] += c
                moved += c != 0.0
        o.sweep(u, f, 1, colour)
        assert np.array_equal(u, expect), (colour, float(np.max(np.abs(u - expect))))
        if colours == 4:
            # the in-place (Gauss-Seidel) order would differ: solving one pixel after its same-colour
            # neighbour two columns away has moved gives another correction somewhere
            gs = before.copy()
            for i in range(H):
                for j in range(W):
                    if 2 * (i % 2) + (j % 2) == colour:
                        gs[i, j] += o.local_solve(gs, f, (i, i + 1, j, j + 1)).c
            changed_neighbour += int(not np.array_equal(gs, expect))
    assert moved > H * W // 4
    if colours == 4:
        assert changed_neighbour == 4


def test_p5_four_colour_fine_level_reports_increases(orc):
    """At b = 1 with four colours a sweep is Jacobi-within-colour; every individual block step is
    non-increasing, and the whole-solve energy still decreases overall."""
    f, _ = noisy_image(32, 32, 4, 0.1)
    o = orc.Oracle(32, 32, 20.0, 0)
    u = f.copy()
    n, trace = o.solve(u, f, rel_tol=0.0, max_vcycles=5)
    assert trace[-1] < trace[0]
    assert np.all(np.diff(trace) <= 1e-9 * trace[0])


def test_p6_constant_fixed_point(orc):
    """P6: a constant image is a fixed point (F = 0, so rho = 0 and every c = 0): u stays bitwise f."""
    for kind in (0, 1):
        f = np.full((17, 23), 0.625)
        o = orc.Oracle(17, 23, 20.0, kind)
        u = f.copy()
        o.solve(u, f, rel_tol=0.0, max_vcycles=3)
        assert np.array_equal(u, f)


@pytest.mark.parametrize("kind", [0, 1])
def test_p7_invariances(orc, kind):
    """P7: f -> f + t gives u -> u + t; f -> -f gives u -> -u (|kappa| and the data term are even)."""
    f, _ = noisy_image(16, 16, 21, 0.1)
    o = orc.Oracle(16, 16, 20.0, kind)
    u = f.copy()
    o.solve(u, f, rel_tol=0.0, max_vcycles=3)
    t = 0.25
    f2 = f + t
    u2 = f2.copy()
    o.solve(u2, f2, rel_tol=0.0, max_vcycles=3)
    assert np.max(np.abs((u2 - t) - u)) < 1e-9
    f3 = -f
    u3 = f3.copy()
    o.solve(u3, f3, rel_tol=0.0, max_vcycles=3)
    assert np.max(np.abs(u3 + u)) < 1e-9


def test_p8_large_alpha_limit(orc):
    """P8: alpha -> infinity pins u to f."""
    f, _ = noisy_image(16, 16, 8, 0.1)
    for kind in (0, 1):
        o = orc.Oracle(16, 16, 1e10, kind)
        u = f.copy()
        o.solve(u, f, rel_tol=0.0, max_vcycles=2)
        assert np.max(np.abs(u - f)) < 1e-6


def test_energy_decreases_and_denoises(orc):
    """End-to-end: the energy trace is non-increasing and the result is closer to the clean image."""
    f, g = noisy_image(48, 48, 2, 0.08)
    o = orc.Oracle(48, 48, 20.0, 0, fine_colours=9)
    u = f.copy()
    n, trace = o.solve(u, f, rel_tol=1e-6, max_vcycles=60)
    assert np.all(np.diff(trace) <= 1e-10 * trace[0])
    assert np.sqrt(np.mean((u - g) ** 2)) < np.sqrt(np.mean((f - g) ** 2))


def test_round_f32_state(orc):
    """The float-state option keeps every state value representable in float32."""
    f, _ = noisy_image(16, 16, 9, 0.1, dtype=np.float32)
    f = f.astype(np.float64)
    o = orc.Oracle(16, 16, 20.0, 0, round_f32=True)
    u = f.copy()
    o.solve(u, f, rel_tol=0.0, max_vcycles=2)
    assert np.array_equal(u, u.astype(np.float32).astype(np.float64))


def test_accept_rule_rejects_worse_candidates(orc):
    """With a deliberately coarse search (3 samples, no bisection) on a near-converged state, some
    blocks' best candidate is worse than c = 0; the accept rule must return 0 there and the energy
    must still not increase."""
    f, _ = noisy_image(24, 24, 13, 0.08)
    o = orc.Oracle(24, 24, 20.0, 0)
    u = f.copy()
    o.solve(u, f, rel_tol=0.0, max_vcycles=4)
    coarse = orc.Oracle(24, 24, 20.0, 0, samples=2, bisections=0)
    rejected = 0
    for level in (1, 2, 3):
        for p, q, bnd in _blocks(coarse, level):
            info = coarse.local_solve(u, f, bnd)
            eta = 1e-12 * (1 + info.K0 + 0.5 * 20.0 * info.s * info.fs ** 2)
            if info.delta >= -eta:
                assert info.accepted == 0 and info.c == 0.0
                rejected += 1
            else:
                assert info.accepted == 1 and info.c == info.c_tilde
    assert rejected > 0
    E0 = coarse.energy(u, f)
    for level in (2, 3):
        for colour in range(4):
            coarse.sweep(u, f, level, colour)
            E1 = coarse.energy(u, f)
            assert E1 <= E0 + 1e-10 * E0
            E0 = E1


@pytest.mark.parametrize("kind", [0, 1])
def test_accept_rule_keeps_zero_on_unresolved_ties(orc, kind):
    """A correction whose gain is below the rounding margin eta = 1e-12 (1 + V(0)) of the computed
    local change is a tie with c = 0 that FP64 cannot resolve; the accept rule keeps c = 0 there.
    Built on a bowl whose curvature stays away from zero (so V is smooth at the optimum, not on a
    kink of |kappa|): each pixel block is first moved to its own optimum, then displaced by
    d = 2e-8, so that the solver's best correction is about -d with a gain of about V'' d^2 / 2
    (a few 1e-15), far below eta but still negative."""
    H, W = 16, 16
    ii, jj = np.mgrid[0:H, 0:W].astype(float)
    f = 0.02 * ((ii - 7.3) ** 2 + (jj - 8.1) ** 2) + 0.01 * np.sin(0.7 * ii + 0.4 * jj)
    o = orc.Oracle(H, W, 20.0, kind)
    u = f.copy()
    n_ties = 0
    for i in range(2, H - 2, 3):
        for j in range(2, W - 2, 3):
            bnd = (i, i + 1, j, j + 1)
            x = u.copy()
            first = o.local_solve(x, f, bnd)
            x[i, j] += first.c_tilde + 2e-8
            info = o.local_solve(x, f, bnd)
            eta = 1e-12 * (1 + info.K0 + 0.5 * 20.0 * info.s * info.fs ** 2)
            if -eta <= info.delta < 0.0 and info.c_tilde != 0.0:
                assert info.accepted == 0 and info.c == 0.0, (i, j, info.delta, eta)
                n_ties += 1
            else:
                assert info.accepted == (info.delta < -eta)
    assert n_ties >= 12, n_ties


@pytest.mark.parametrize("kind", [0, 1])
def test_full_cycle_monotone_and_fixed_point(orc, kind):
    """Full V-cycle (Section 2.2: fine to coarse, then back to the finest level): with nine fine
    colours every sweep is non-increasing, so one full cycle ends at or below the half cycle it
    starts with; a constant image stays bitwise fixed; with J = 1 there is nothing to go back
    through and the two cycles agree bitwise."""
    H, W = 26, 21
    f, _ = noisy_image(H, W, 5, 0.08)
    half = orc.Oracle(H, W, 20.0, kind, fine_colours=9)
    full = orc.Oracle(H, W, 20.0, kind, fine_colours=9, cycle=1)
    uh, uf = f.copy(), f.copy()
    half.vcycle(uh, f)
    full.vcycle(uf, f)
    assert full.energy(uf, f) <= half.energy(uh, f) + 1e-10 * (1 + half.energy(uh, f))
    assert not np.array_equal(uh, uf)
    c = np.full((H, W), 0.375)
    u = c.copy()
    full.vcycle(u, c)
    assert np.array_equal(u, c)
    one_h = orc.Oracle(H, W, 20.0, kind, levels=1)
    one_f = orc.Oracle(H, W, 20.0, kind, levels=1, cycle=1)
    a, b = f.copy(), f.copy()
    one_h.vcycle(a, f)
    one_f.vcycle(b, f)
    assert np.array_equal(a, b)


def test_energy_stop_rule_is_the_first_small_change(orc):
    """The relative energy-change rule of Section 4 (|E_l - E_{l-1}| < tol |E_l|, E_0 = F(u_0); an
    unchanged energy also stops): replayed cycle by cycle with the energies of the replay, for the
    half and the full cycle; the solve stops at the first small change, its trace is the replay's and
    its state equals the replay's bitwise.  A rule with no step small enough runs to the cap."""
    H, W = 30, 27
    f, _ = noisy_image(H, W, 8, 0.1)
    for cycle in (0, 1):
        o = orc.Oracle(H, W, 20.0, 0, cycle=cycle)
        for tol in (3e-3, 2e-4):
            u = f.copy()
            n, trace = o.solve(u, f, rel_tol=tol, max_vcycles=60)
            assert 2 <= n < 60 and len(trace) == n + 1, (cycle, tol, n)
            v = f.copy()
            e_prev = o.energy(v, f)
            assert trace[0] == e_prev
            for l in range(1, n + 1):
                o.vcycle(v, f)
                e = o.energy(v, f)
                assert trace[l] == e
                small = e == e_prev or abs(e - e_prev) < tol * abs(e)
                assert small == (l == n), (cycle, tol, l, n, e, e_prev)
                e_prev = e
            assert np.array_equal(u, v)
    # tol 0: exactly the requested count
    o = orc.Oracle(H, W, 20.0, 0)
    n, trace = o.solve(f.copy(), f, rel_tol=0.0, max_vcycles=5)
    assert n == 5 and len(trace) == 6
    # a constant image: E = 0 throughout, the unchanged energy stops after one cycle
    c = np.full((H, W), 0.5)
    n, trace = o.solve(c.copy(), c, rel_tol=1e-6, max_vcycles=10)
    assert n == 1 and trace[0] == 0.0 and trace[1] == 0.0


def test_relerr_stop_rule_is_the_first_small_step(orc):
    """The relErr(u) rule of Section 4 (||u_l - u_{l-1}|| < tol ||u_l||) stops at the first V-cycle
    whose step is small: replayed cycle by cycle, with the norms taken by numpy."""
    H, W = 30, 27
    f, _ = noisy_image(H, W, 8, 0.1)
    for cycle in (0, 1):
        o = orc.Oracle(H, W, 20.0, 0, cycle=cycle)
        tol = 3e-3
        u = f.copy()
        n, trace = o.solve_rule(u, f, tol, max_vcycles=60, stop=1)
        assert 1 <= n < 60 and len(trace) == n + 1
        v = f.copy()
        for l in range(1, n + 1):
            prev = v.copy()
            o.vcycle(v, f)
            small = np.linalg.norm(v - prev) < tol * np.linalg.norm(v)
            assert small == (l == n), (cycle, l, n)
        assert np.array_equal(u, v)
    # a constant image does not move: relErr = 0 after the first cycle
    c = np.full((H, W), 0.5)
    o = orc.Oracle(H, W, 20.0, 1)
    n, _ = o.solve_rule(c.copy(), c, 1e-9, max_vcycles=10, stop=1)
    assert n == 1


def test_paper_block_schedule_geometry(orc):
    """Section 2.2's hierarchy: patch side 2^j - 1 and m_j = ceil(m / (2^j - 1)) patches along a
    side of m pixels.  The expected values are worked by hand for a 100 x 37 image; the nested
    power-of-two schedule is the default, and at j = 1 both are single pixels."""
    o = orc.Oracle(100, 37, 20.0, 0, levels=6, schedule=1)
    assert [o.block_side(j) for j in range(1, 7)] == [1, 3, 7, 15, 31, 63]
    assert [o.grid(j) for j in range(1, 7)] == [(100, 37), (34, 13), (15, 6), (7, 3), (4, 2), (2, 1)]
    o0 = orc.Oracle(100, 37, 20.0, 0, levels=6)
    assert [o0.block_side(j) for j in range(1, 7)] == [1, 2, 4, 8, 16, 32]
    assert [o0.grid(j) for j in range(1, 7)] == [(100, 37), (50, 19), (25, 10), (13, 5), (7, 3), (4, 2)]


@pytest.mark.parametrize("kind", [0, 1])
def test_paper_schedule_sweeps_move_whole_patches(orc, kind):
    """With the 2^j - 1 schedule a colour sweep at level j adds one constant to every patch of side
    2^j - 1 (clipped at the right and bottom) whose colour 2 (P mod 2) + (Q mod 2) is the sweep's,
    and leaves every other pixel bitwise alone; each constant is the local solver's on that patch,
    from the state before the sweep.  The patch side is written here, not taken from the oracle."""
    H, W = 23, 19
    f, _ = noisy_image(H, W, 21, 0.1)
    o = orc.Oracle(H, W, 20.0, kind, levels=3, schedule=1)
    u = f.copy()
    o.vcycle(u, f)
    moved = 0
    for j in (2, 3):
        b = 2 ** j - 1
        for colour in range(4):
            before = u.copy()
            expect = u.copy()
            for P in range(-(-H // b)):
                for Q in range(-(-W // b)):
                    if 2 * (P % 2) + (Q % 2) != colour:
                        continue
                    bnd = (P * b, min(P * b + b, H), Q * b, min(Q * b + b, W))
                    c = o.local_solve(before, f, bnd).c
                    expect[bnd[0]:bnd[1], bnd[2]:bnd[3]] += c
                    moved += c != 0.0
            o.sweep(u, f, j, colour)
            assert np.array_equal(u, expect), (j, colour)
    assert moved > 20


@pytest.mark.parametrize("kind", [0, 1])
def test_paper_schedule_sweeps_monotone_and_separable(orc, kind):
    """P5 + P9 on the 2^j - 1 patches: with nine fine colours every colour sweep changes F by the
    sum of its patches' local changes, none positive (same-colour patches are at least one patch
    apart, so their rings do not meet); a full solve never raises F."""
    H, W = 26, 22
    f, _ = noisy_image(H, W, 12, 0.08)
    o = orc.Oracle(H, W, 20.0, kind, fine_colours=9, levels=4, schedule=1)
    u = f.copy()
    for level in range(1, o.levels + 1):
        for colour in range(o.num_colours(level)):
            E0 = o.energy(u, f)
            deltas = []
            for p, q, bnd in _blocks(o, level):
                if o.colour_of(level, p, q) != colour:
                    continue
                info = o.local_solve(u, f, bnd)
                deltas.append(info.delta if info.accepted else 0.0)
            o.sweep(u, f, level, colour)
            E1 = o.energy(u, f)
            assert abs((E1 - E0) - sum(deltas)) < 1e-10 * (1 + E0), (level, colour)
            assert E1 <= E0 + 1e-10 * (1 + E0)
    v = f.copy()
    _, trace = o.solve(v, f, rel_tol=0.0, max_vcycles=4)
    assert np.all(np.diff(trace) <= 1e-10 * trace[0])


def test_paper_schedule_single_level_equals_pixel_level(orc):
    """At J = 1 both schedules are the pixel level: one V-cycle agrees bitwise."""
    f, _ = noisy_image(19, 24, 3, 0.1)
    a, b = f.copy(), f.copy()
    orc.Oracle(19, 24, 20.0, 0, levels=1).vcycle(a, f)
    orc.Oracle(19, 24, 20.0, 0, levels=1, schedule=1).vcycle(b, f)
    assert np.array_equal(a, b)
    assert not np.array_equal(a, f)
