"""Pins of the reconstruction oracle (Section 5) against what the mathematics fixes,
independently of the oracle's code:

* A^T is the transpose of A, both built column by column as explicit matrices;
* the blur weights are the normalised Gaussian, and A keeps a constant away from the border;
* the corrections of one colour are the stationary point (and minimiser) of the paper's
  quadratic subproblem, checked by finite differences and random perturbations of the
  objective evaluated from its definition;
* with the identity operator the system is diagonal and has a closed form;
* with alpha -> 0 a colour sweep cannot raise the data term (c = 0 is feasible);
* the energy is its definition evaluated with scipy's correlation.
"""
import math

import numpy as np
import pytest
from scipy.ndimage import correlate

from oracle.oracle import curvature_map
from oracle.recon_oracle import ReconOracle, apply_A, apply_At, blur_weights


def _img(h, w, seed, scale=1.0):
    return scale * np.random.default_rng(seed).standard_normal((h, w))


def test_adjoint_is_the_transpose():
    h, w = 7, 6
    wts = blur_weights(1.3)
    n = h * w
    A = np.empty((n, n))
    At = np.empty((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = apply_A(e.reshape(h, w), wts).ravel()
        At[:, k] = apply_At(e.reshape(h, w), wts).ravel()
    assert np.allclose(At, A.T, rtol=0, atol=1e-15)
    # and A matches scipy's correlation with a zero boundary
    u = _img(h, w, 1)
    assert np.allclose(apply_A(u, wts), correlate(u, wts, mode="constant", cval=0.0), rtol=0, atol=1e-14)


def test_blur_weights():
    for sigma in (0.7, 1.0, 2.0):
        wts = blur_weights(sigma)
        assert wts.shape == (5, 5)
        assert wts.sum() == pytest.approx(1.0, abs=1e-15)
        assert wts[2, 3] / wts[2, 2] == pytest.approx(math.exp(-1.0 / (2 * sigma * sigma)), rel=1e-14)
        assert wts[0, 0] / wts[2, 2] == pytest.approx(math.exp(-8.0 / (2 * sigma * sigma)), rel=1e-14)
        const = np.full((12, 12), 0.37)
        assert np.allclose(apply_A(const, wts)[2:-2, 2:-2], 0.37, rtol=0, atol=1e-15)


def _objective(o, u, b, level, ps, c, d):
    v = u.copy()
    for (p, q), ci in zip(ps, c):
        r0, r1, c0, c1 = o.fbs.block_bounds(level, p, q)
        v[r0:r1, c0:c1] += ci
    res = correlate(v, o.wts, mode="constant", cval=0.0) - b
    return 0.5 * float(np.sum(res * res)) + o.alpha * float(np.sum((np.asarray(c) - d) ** 2))


@pytest.mark.parametrize("level,colour", [(1, 0), (1, 3), (2, 1), (3, 2)])
def test_colour_solution_minimises_the_subproblem(level, colour):
    h, w = 17, 15
    o = ReconOracle(h, w, alpha=0.03, sigma_a=1.0, levels=3)
    u = _img(h, w, 2, 0.3)
    b = _img(h, w, 3, 0.3)
    ps, G, r, d = o.system(u, b, level, colour)
    uu = u.copy()
    cgrid = o.sweep(uu, b, level, colour)
    c = np.array([cgrid[p, q] for p, q in ps])
    q0 = _objective(o, u, b, level, ps, c, d)
    eps = 1e-6
    for i in range(len(c)):
        e = np.zeros_like(c)
        e[i] = eps
        g = (_objective(o, u, b, level, ps, c + e, d) - _objective(o, u, b, level, ps, c - e, d)) / (2 * eps)
        assert abs(g) < 1e-7, (i, g)
    rng = np.random.default_rng(4)
    for _ in range(10):
        assert _objective(o, u, b, level, ps, c + 1e-3 * rng.standard_normal(len(c)), d) > q0


def test_identity_operator_has_a_diagonal_closed_form():
    h, w = 14, 11
    o = ReconOracle(h, w, alpha=0.2, sigma_a=0.05, levels=3)   # weights off the centre underflow to 0
    assert o.wts[2, 2] == 1.0 and o.wts.sum() == 1.0
    u = _img(h, w, 5)
    b = _img(h, w, 6)
    for level, colour in [(1, 1), (2, 0), (3, 3)]:
        ps, _, _, d = o.system(u, b, level, colour)
        uu = u.copy()
        cgrid = o.sweep(uu, b, level, colour)
        for (p, q), di in zip(ps, d):
            r0, r1, c0, c1 = o.fbs.block_bounds(level, p, q)
            s = (r1 - r0) * (c1 - c0)
            expect = (np.sum(b[r0:r1, c0:c1] - u[r0:r1, c0:c1]) + 2 * o.alpha * di) / (s + 2 * o.alpha)
            assert cgrid[p, q] == pytest.approx(expect, rel=1e-12, abs=1e-14)


def test_data_term_cannot_rise_without_regularisation():
    h, w = 16, 16
    o = ReconOracle(h, w, alpha=1e-12, sigma_a=1.2, levels=3)
    g = _img(h, w, 7, 0.5)
    b = apply_A(g, o.wts) + 0.05 * _img(h, w, 8)
    u = b.copy()
    data = lambda v: 0.5 * float(np.sum((apply_A(v, o.wts) - b) ** 2))
    prev = data(u)
    for level in (1, 2, 3):
        for colour in range(4):
            o.sweep(u, b, level, colour)
            cur = data(u)
            assert cur <= prev + 1e-12
            prev = cur


def test_energy_definition():
    h, w = 13, 19
    o = ReconOracle(h, w, alpha=0.07, sigma_a=1.0)
    u = _img(h, w, 9, 0.4)
    b = _img(h, w, 10, 0.4)
    res = correlate(u, o.wts, mode="constant", cval=0.0) - b
    expect = 0.5 * np.sum(res ** 2) + 0.07 * np.sum(np.abs(curvature_map(0, u)))
    assert o.energy(u, b) == pytest.approx(expect, rel=1e-13)
