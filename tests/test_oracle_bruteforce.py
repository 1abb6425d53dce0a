"""P3 + P4 at full scale: the oracle's local solver against brute-force minimisation of the local
energy on 100 seeded 8x8 images, mean and Gaussian curvature, block sides 1, 2 and 4 (levels 1-3),
every block of every level.

The brute force is independent of the oracle's search: a dense grid of V(c) = K(c) + alpha s/2
(c - f*)^2 over three bracket widths on each side of f*, then six zoom passes around the best grid
point.  It uses only the oracle's K(c) (the ring sum, itself pinned by the whole-image identity P2).
Asserted per block:
  * P3: the brute-force minimiser lies inside [f* - rho, f* + rho];
  * P4: V at the solver's candidate is within 1e-9 (1 + K(0)) of the brute-force minimum, and the
    candidate lies no farther from the brute-force minimiser than the grid points whose V is within
    that tolerance do (or 1e-6): it is in the same basin, and where the minimiser is unique (those
    points lie within 1e-4) that pins its position;
  * the accept rule: an applied correction lowers the local energy by more than eta = 1e-12 (1 + V(0)),
    a rejected one is 0.
"""
import numpy as np
import pytest

from synth import noisy_image

N_IMAGES = 100
CHUNK = 25


def _V(o, u, bnd, fs, a, cs):
    return o.ring_K_many(u, bnd, cs) + 0.5 * a * (cs - fs) ** 2


def _brute(o, u, bnd, fs, a, lo, hi, n=3001):
    cs = np.linspace(lo, hi, n)
    v = _V(o, u, bnd, fs, a, cs)
    k = int(np.argmin(v))
    best_c, best_v = cs[k], v[k]
    pts, vals = [cs], [v]
    span = (hi - lo) / (n - 1)
    for _ in range(6):
        cz = np.linspace(best_c - span, best_c + span, 201)
        vz = _V(o, u, bnd, fs, a, cz)
        pts.append(cz)
        vals.append(vz)
        k = int(np.argmin(vz))
        if vz[k] <= best_v:
            best_c, best_v = cz[k], vz[k]
        span = 2 * span / 200
    return best_c, best_v, np.concatenate(pts), np.concatenate(vals)


@pytest.mark.parametrize("first", range(0, N_IMAGES, CHUNK))
@pytest.mark.parametrize("kind", [0, 1])
def test_p3_p4_bruteforce_100_images(orc, kind, first):
    n_blocks = n_unique = n_accepted = 0
    worst_gap = 0.0
    for seed in range(first, first + CHUNK):
        f, _ = noisy_image(8, 8, 1000 + seed, 0.1)
        rng = np.random.default_rng(5000 + seed)
        u = f + 0.08 * rng.standard_normal(f.shape)
        o = orc.Oracle(8, 8, 20.0, kind)
        for level in (1, 2, 3):
            m, n = o.grid(level)
            for p in range(m):
                for q in range(n):
                    bnd = o.block_bounds(level, p, q)
                    info = o.local_solve(u, f, bnd)
                    fs, s, rho, K0 = info.fs, info.s, info.rho, info.K0
                    a = 20.0 * s
                    wide = max(rho, 1e-3)
                    c_bf, v_bf, pts, vals = _brute(o, u, bnd, fs, a, fs - 3 * wide, fs + 3 * wide)
                    # P3
                    assert abs(c_bf - fs) <= rho + 2e-3 * wide, (seed, level, p, q, c_bf, fs, rho)
                    # P4: value
                    tol_v = 1e-9 * (1 + K0)
                    v_alg = float(_V(o, u, bnd, fs, a, np.array([info.c_tilde]))[0])
                    gap = v_alg - v_bf
                    worst_gap = max(worst_gap, gap / (1 + K0))
                    assert gap <= tol_v, (seed, level, p, q, v_alg, v_bf, info.c_tilde, c_bf)
                    # P4: position.  D = how far from the brute-force minimiser V stays within the
                    # value tolerance; the candidate must lie within D of it (same basin), and where
                    # the minimiser is unique (D <= 1e-4) that is a position check
                    near = pts[vals <= v_bf + tol_v]
                    D = float(np.max(np.abs(near - c_bf)))
                    n_unique += D <= 1e-4
                    assert abs(info.c_tilde - c_bf) <= max(D, 1e-6) + 1e-9 * wide, \
                        (seed, level, p, q, info.c_tilde, c_bf, D)
                    # accept rule
                    eta = 1e-12 * (1 + K0 + 0.5 * a * fs * fs)
                    if info.accepted:
                        assert info.delta < -eta and info.c == info.c_tilde
                        n_accepted += 1
                    else:
                        assert info.c == 0.0 and info.delta >= -eta
                    n_blocks += 1
    assert n_blocks == CHUNK * (64 + 16 + 4)
    print(f"kind {kind} images {first}-{first + CHUNK - 1}: {n_blocks} blocks, unique minimiser in "
          f"{n_unique}, accepted {n_accepted}, worst V gap {worst_gap:.2e} (1 + K0)")
    assert n_unique > n_blocks // 2
