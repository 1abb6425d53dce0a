"""Seeded piecewise-smooth test images (stand-ins for the paper's natural images).

The paper denoises natural photographs (Section 4, the test-image figure and the
30-image study) that are not available here.  These generators produce images of
the same sizes with the structure the method is built for: piecewise-smooth
surfaces with sharp edges plus i.i.d. Gaussian noise.

Recipe (all draws from ``numpy.random.Generator(PCG64(seed))`` in this order):

1. ramp  g = a0 + ax * x / W + ay * y / H,  a0 ~ U[0, 1], ax, ay ~ U[-0.5, 0.5]
   (x = column index, y = row index);
2. ``n_shapes`` shapes painted in order (later ones overwrite earlier ones).
   Each is a disc with probability 1/2 (radius ~ U[0.05, 0.25] * min(H, W)),
   otherwise an axis-aligned rectangle (half sizes ~ U[0.05, 0.25] * (W, H));
   centre ~ U over the image, intensity ~ U[0, 1].  A pixel belongs to a shape
   when its centre (x + 1/2, y + 1/2) does;
3. clip g to [0, 1];
4. f = g + sigma * N(0, 1), not clipped.
"""
from __future__ import annotations

import numpy as np

BATCH_SIZES = (128, 192, 256, 384, 512, 768, 1024)


def piecewise_smooth(height: int, width: int, seed: int, n_shapes: int = 8) -> tuple[np.ndarray, np.random.Generator]:
    """Return (ground truth g in [0,1] as float64 HxW, the generator after drawing g)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a0 = rng.uniform(0.0, 1.0)
    ax, ay = rng.uniform(-0.5, 0.5, size=2)
    y = np.arange(height, dtype=np.float64)[:, None]
    x = np.arange(width, dtype=np.float64)[None, :]
    g = a0 + ax * x / width + ay * y / height
    g = np.broadcast_to(g, (height, width)).copy()
    yc = y + 0.5
    xc = x + 0.5
    for _ in range(n_shapes):
        is_disc = rng.uniform() < 0.5
        if is_disc:
            r = rng.uniform(0.05, 0.25) * min(height, width)
            cx = rng.uniform(0.0, width)
            cy = rng.uniform(0.0, height)
            val = rng.uniform(0.0, 1.0)
            mask = (xc - cx) ** 2 + (yc - cy) ** 2 <= r * r
        else:
            hx = rng.uniform(0.05, 0.25) * width
            hy = rng.uniform(0.05, 0.25) * height
            cx = rng.uniform(0.0, width)
            cy = rng.uniform(0.0, height)
            val = rng.uniform(0.0, 1.0)
            mask = (np.abs(xc - cx) <= hx) & (np.abs(yc - cy) <= hy)
        g[np.broadcast_to(mask, (height, width))] = val
    np.clip(g, 0.0, 1.0, out=g)
    return g, rng


def noisy_image(height: int, width: int, seed: int, sigma: float, n_shapes: int = 8,
                dtype=np.float64) -> tuple[np.ndarray, np.ndarray]:
    """Return (f, g): the noisy observation and its clean ground truth.

    ``dtype=np.float32`` rounds f to single precision; the float64 promotion of
    that array is then the exact input a double-precision reference receives.
    """
    g, rng = piecewise_smooth(height, width, seed, n_shapes)
    f = g + sigma * rng.standard_normal((height, width))
    return np.ascontiguousarray(f.astype(dtype)), g


def batch_specs(n_images: int = 256, seed: int = 0) -> list[dict]:
    """Per-image settings for the mixed-size batch workload.

    Height and width are drawn independently from ``BATCH_SIZES`` (so shapes such
    as 512x1024 occur), sigma ~ U[0.03, 0.12], alpha from {10, 20, 40}, curvature
    kind from {0 (mean), 1 (Gaussian)}; image i uses image seed 1000 + i.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    specs = []
    for i in range(n_images):
        h = int(rng.choice(BATCH_SIZES))
        w = int(rng.choice(BATCH_SIZES))
        sigma = float(rng.uniform(0.03, 0.12))
        alpha = float(rng.choice([10.0, 20.0, 40.0]))
        kind = int(rng.integers(0, 2))
        specs.append(dict(height=h, width=w, sigma=sigma, alpha=alpha, kind=kind, seed=1000 + i))
    return specs
