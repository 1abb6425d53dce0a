"""Plain FP64 oracle of the multigrid reconstruction step (Section 5): recover u from
b = A u + noise by minimising 1/2 ||A u - b||^2 + alpha sum |H(u)|.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and the benchmark's
CPU-baseline leg may import this module; it shares nothing with the HIP path.

What it computes (readings named R..):

* A (R21): the paper's operators (Radon, Fourier) need phantoms and data that are not
  available; a 5 x 5 Gaussian blur stands in for them: (A u)(p) = sum_q w(q - p) u(q) over the
  image, w the normalised Gaussian of width sigma_A, positions outside the image contributing
  nothing (zero boundary).  A^T is the same sum with the offset negated.
* Patches and colours: the paper's schedule (side 2^j - 1, anchored at the top-left pixel,
  four colours 2 (p mod 2) + (q mod 2)), as for the paper's own local step.
* Per colour k of level j (Section 5): with phi_i the indicator of patch i and d_i the
  tangent-plane estimate of Proposition 1 (the mean of the signed distances from the patch
  centre to its 2^(j+2) planes, R22), the corrections of all patches of the colour solve
      (G + 2 alpha I) c = r,   G_il = <A phi_i, A phi_l>,   r_i = <b - A u, A phi_i> + 2 alpha d_i,
  the stationary point of 1/2 ||A(u + sum c_i phi_i) - b||^2 + alpha sum (c_i - d_i)^2; the oracle
  builds G explicitly and solves the system exactly; then u <- u + sum c_i phi_i.
* V-cycle: levels 1..J fine to coarse, four colours each (the half V-cycle).
* Energy: 1/2 ||A u - b||^2 + alpha sum |kappa_MC(u)| with the discrete mean curvature of the
  denoising model (replicated ghosts, 3 x 3 central differences).
"""
from __future__ import annotations

import math

import numpy as np

from .oracle import FbsOracle, curvature_map

RADIUS = 2   # 5 x 5 blur


def blur_weights(sigma: float) -> np.ndarray:
    """Normalised 5 x 5 Gaussian, w[dy + 2, dx + 2]."""
    w = np.empty((2 * RADIUS + 1, 2 * RADIUS + 1))
    for dy in range(-RADIUS, RADIUS + 1):
        for dx in range(-RADIUS, RADIUS + 1):
            w[dy + RADIUS, dx + RADIUS] = math.exp(-(dx * dx + dy * dy) / (2.0 * sigma * sigma))
    return w / w.sum()


def apply_A(u: np.ndarray, w: np.ndarray) -> np.ndarray:
    """(A u)(p) = sum over offsets o of w[o] u(p + o), zero outside the image."""
    h, wd = u.shape
    out = np.zeros((h, wd))
    pad = np.zeros((h + 2 * RADIUS, wd + 2 * RADIUS))
    pad[RADIUS:RADIUS + h, RADIUS:RADIUS + wd] = u
    for dy in range(-RADIUS, RADIUS + 1):
        for dx in range(-RADIUS, RADIUS + 1):
            out += w[dy + RADIUS, dx + RADIUS] * pad[RADIUS + dy:RADIUS + dy + h, RADIUS + dx:RADIUS + dx + wd]
    return out


def apply_At(v: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Adjoint of apply_A: (A^T v)(q) = sum over offsets o of w[o] v(q - o), zero outside."""
    return apply_A(v, w[::-1, ::-1])


class ReconOracle:
    def __init__(self, height: int, width: int, alpha: float, sigma_a: float = 1.0, levels: int = 3,
                 round_f32: bool = False):
        self.h, self.w, self.alpha, self.levels = height, width, float(alpha), levels
        self.round_f32 = round_f32   # round the state to float after each update
        self.wts = blur_weights(sigma_a)
        # the tangent-plane estimate and the patch geometry of the paper's local step
        self.fbs = FbsOracle(height, width, 1.0, 0, levels=levels)

    def grid(self, level: int):
        return self.fbs.grid(level)

    def patches(self, level: int, colour: int):
        mj, nj = self.grid(level)
        return [(p, q) for p in range(mj) for q in range(nj) if 2 * (p % 2) + (q % 2) == colour]

    def indicator(self, level: int, p: int, q: int) -> np.ndarray:
        r0, r1, c0, c1 = self.fbs.block_bounds(level, p, q)
        phi = np.zeros((self.h, self.w))
        phi[r0:r1, c0:c1] = 1.0
        return phi

    def system(self, u: np.ndarray, b: np.ndarray, level: int, colour: int):
        """(patches, G, r, d) of the coupled problem of one colour."""
        ps = self.patches(level, colour)
        aphi = [apply_A(self.indicator(level, p, q), self.wts) for p, q in ps]
        resid = b - apply_A(u, self.wts)
        n = len(ps)
        G = np.empty((n, n))
        for i in range(n):
            for l in range(i, n):
                G[i, l] = G[l, i] = float(np.sum(aphi[i] * aphi[l]))
        d = np.array([self.fbs.estimate(u, level, p, q) for p, q in ps])
        r = np.array([float(np.sum(resid * aphi[i])) for i in range(n)]) + 2.0 * self.alpha * d
        return ps, G, r, d

    def sweep(self, u: np.ndarray, b: np.ndarray, level: int, colour: int) -> np.ndarray:
        """In-place colour sweep; returns the corrections on the level's patch grid (0 elsewhere)."""
        ps, G, r, _ = self.system(u, b, level, colour)
        cgrid = np.zeros(self.grid(level))
        if not ps:
            return cgrid
        c = np.linalg.solve(G + 2.0 * self.alpha * np.eye(len(ps)), r)
        for (p, q), ci in zip(ps, c):
            r0, r1, c0, c1 = self.fbs.block_bounds(level, p, q)
            u[r0:r1, c0:c1] += ci
            if self.round_f32:
                u[r0:r1, c0:c1] = u[r0:r1, c0:c1].astype(np.float32).astype(np.float64)
            cgrid[p, q] = ci
        return cgrid

    def vcycle(self, u: np.ndarray, b: np.ndarray) -> None:
        for level in range(1, self.levels + 1):
            for colour in range(4):
                self.sweep(u, b, level, colour)

    def energy(self, u: np.ndarray, b: np.ndarray) -> float:
        res = apply_A(u, self.wts) - b
        return 0.5 * float(np.sum(res * res)) + self.alpha * float(np.sum(np.abs(curvature_map(0, u))))
