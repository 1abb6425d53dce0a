"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module draws images and per-image settings only; it holds none of the
method's arithmetic (no curvature, no energy, no solver step).
"""
from .cnn_init import CHANNELS, init_params, n_params  # noqa: F401
from .images import (  # noqa: F401
    piecewise_smooth,
    noisy_image,
    batch_specs,
    BATCH_SIZES,
)
