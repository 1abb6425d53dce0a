"""Pins of the FP64 CNN reference: convolution against scipy's correlate2d (single channel),
the transposed convolution as the exact adjoint (<conv x, y> = <x, conv^T y>), gradients against
central finite differences of the loss, the first Adam step in closed form, bfloat16 rounding
against hand-computed values."""
import numpy as np
import pytest
from scipy.signal import correlate2d

from oracle import cnn_ref
from synth import init_params, n_params


def test_param_count():
    assert n_params() == 37601
    assert init_params(0).size == 37601


def test_conv_matches_scipy_correlate_single_channel():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 7, 9, 1))
    W = rng.standard_normal((3, 3, 1, 1))
    b = np.array([0.3])
    y = cnn_ref.conv(x, W, b)
    ref = correlate2d(x[0, :, :, 0], W[:, :, 0, 0], mode="same", boundary="fill", fillvalue=0.0) + 0.3
    assert np.allclose(y[0, :, :, 0], ref, atol=1e-13)


def test_conv_channel_mixing_is_sum_of_single_channel_correlations():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 5, 6, 3))
    W = rng.standard_normal((3, 3, 3, 4))
    y = cnn_ref.conv(x, W, np.zeros(4))
    for n in range(2):
        for o in range(4):
            ref = sum(correlate2d(x[n, :, :, c], W[:, :, c, o], mode="same") for c in range(3))
            assert np.allclose(y[n, :, :, o], ref, atol=1e-12)


def test_transpose_is_adjoint():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 5, 4))
    dy = rng.standard_normal((2, 6, 5, 3))
    W = rng.standard_normal((3, 3, 4, 3))
    lhs = np.sum(cnn_ref.conv(x, W, np.zeros(3)) * dy)
    rhs = np.sum(x * cnn_ref.conv_transpose_taps(dy, W))
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    # weight gradient is the adjoint in W
    dW = cnn_ref.weight_grad(x, dy)
    V = rng.standard_normal(W.shape)
    assert abs(np.sum(cnn_ref.conv(x, V, np.zeros(3)) * dy) - np.sum(V * dW)) < 1e-10


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(3)
    f = rng.uniform(0, 1, (2, 6, 7))
    target = f + 0.05 * rng.standard_normal(f.shape)
    p = init_params(5) * 3.0  # larger weights so that ReLUs switch inside the net
    p[-1] = 0.01
    loss, g = cnn_ref.loss_and_grad(p, f, target)
    idx = rng.choice(p.size, size=60, replace=False)
    idx = np.concatenate([idx, np.arange(p.size - 40, p.size)])  # include the last layers and biases
    h = 1e-6
    for k in idx:
        e = np.zeros_like(p)
        e[k] = h
        fd = (cnn_ref.loss_and_grad(p + e, f, target)[0] - cnn_ref.loss_and_grad(p - e, f, target)[0]) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1e-4, abs(fd)) + 1e-9, (k, fd, g[k])


def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3])
    w, m, v = cnn_ref.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    # after one step mhat = g and vhat = g^2, so the step is lr * g / (|g| + eps)
    assert np.allclose(w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_round_bf16_values():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.14159, 0.0, 1.0 + 3 * 2 ** -8])
    r = cnn_ref.round_bf16(x)
    assert r[0] == 1.0
    assert r[1] == 1.0            # tie rounds to even (mantissa 0)
    assert r[2] == 1.0 + 2 ** -7  # 1.0117 rounds up
    assert r[3] == -3.140625
    assert r[4] == 0.0
    assert r[5] == 1.0 + 2 ** -6    # tie between 1 + 2^-7 (odd) and 1 + 2^-6 (even) goes to even
