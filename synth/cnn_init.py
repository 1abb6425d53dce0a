"""Seeded initial parameters of the warm-start CNN (random draws only, no network arithmetic).

Layout of the flat parameter vector (float64 here, float32 on the GPU), layer by layer for
l = 0..5 with channels C = [1, 32, 32, 32, 32, 32, 1]:
    W_l with shape (3, 3, C[l], C[l+1]) in row-major order (ky, kx, c_in, c_out), then
    b_l with shape (C[l+1],).
Weights are He-normal with fan-in 9 * C[l]; the last layer is scaled by 0.1 so that the
initial residual output stays near the identity u = f; biases start at zero.
"""
import numpy as np

CHANNELS = (1, 32, 32, 32, 32, 32, 1)


def n_params() -> int:
    return sum(9 * ci * co + co for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]))


def init_params(seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for l, (ci, co) in enumerate(zip(CHANNELS[:-1], CHANNELS[1:])):
        std = np.sqrt(2.0 / (9 * ci))
        if l == len(CHANNELS) - 2:
            std *= 0.1
        parts.append(rng.standard_normal(9 * ci * co) * std)
        parts.append(np.zeros(co))
    return np.concatenate(parts)
