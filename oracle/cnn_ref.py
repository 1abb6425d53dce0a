"""FP64 NumPy reference of the warm-start CNN (test infrastructure only).

Network: six 3x3 convolutions with zero "same" padding, channels 1 -> 32 -> 32 -> 32 -> 32 -> 32
-> 1, ReLU after the first five, and a residual output u_pred = f + g(f).  Loss: mean squared
error against the multigrid solution u*.  Optimiser: Adam with bias correction.

Every function here is the plain definition: a convolution is a sum over the nine taps of a
channel contraction (numpy matmul per tap), the backward pass is the chain rule written out,
Adam is its published update (Kingma and Ba, 2015, Algorithm 1).  `round_bf16` emulates
bfloat16 storage (round to nearest even) where the GPU stores bfloat16.

Parameter vector layout: see synth/cnn_init.py.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (1, 32, 32, 32, 32, 32, 1)


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float64."""
    f = np.asarray(x, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    bits = ((bits + 0x7FFF + lsb) >> 16) << 16
    return bits.astype(np.uint32).view(np.float32).astype(np.float64)


def unpack(params: np.ndarray):
    """Flat vector -> list of (W (3, 3, ci, co), b (co,))."""
    out, k = [], 0
    for ci, co in zip(CHANNELS[:-1], CHANNELS[1:]):
        W = params[k:k + 9 * ci * co].reshape(3, 3, ci, co)
        k += 9 * ci * co
        b = params[k:k + co]
        k += co
        out.append((W, b))
    assert k == params.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.reshape(-1), b.reshape(-1)]) for W, b in layers])


def conv(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, i, j, o] = b[o] + sum_{ky, kx, c} x[n, i + ky - 1, j + kx - 1, c] W[ky, kx, c, o], zero outside."""
    n, h, w, ci = x.shape
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.broadcast_to(b, (n, h, w, W.shape[3])).copy()
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + w, :] @ W[ky, kx]
    return y


def conv_transpose_taps(dy: np.ndarray, W: np.ndarray) -> np.ndarray:
    """Adjoint of `conv` in x: dx[n, i, j, c] = sum_{ky, kx, o} dy[n, i - ky + 1, j - kx + 1, o] W[ky, kx, c, o]."""
    n, h, w, co = dy.shape
    dyp = np.zeros((n, h + 2, w + 2, co))
    dyp[:, 1:-1, 1:-1, :] = dy
    dx = np.zeros((n, h, w, W.shape[2]))
    for ky in range(3):
        for kx in range(3):
            # dy at (i - ky + 1, j - kx + 1) sits at padded index (i - ky + 2, j - kx + 2)
            dx += dyp[:, 2 - ky:2 - ky + h, 2 - kx:2 - kx + w, :] @ W[ky, kx].T
    return dx


def weight_grad(x: np.ndarray, dy: np.ndarray) -> np.ndarray:
    """dW[ky, kx, c, o] = sum_{n, i, j} x[n, i + ky - 1, j + kx - 1, c] dy[n, i, j, o]."""
    n, h, w, ci = x.shape
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    dW = np.zeros((3, 3, ci, dy.shape[3]))
    for ky in range(3):
        for kx in range(3):
            a = xp[:, ky:ky + h, kx:kx + w, :].reshape(-1, ci)
            dW[ky, kx] = a.T @ dy.reshape(-1, dy.shape[3])
    return dW


def forward(params: np.ndarray, f: np.ndarray, bf16: bool = False, acts_in=None):
    """f: (n, h, w).  Returns (u_pred (n, h, w), activations a_0..a_5 (NHWC)).

    With bf16=True the weights and the stored activations a_1..a_5 are rounded to bfloat16 as
    the GPU stores them.  acts_in (optional list) replaces a_l by a given input before layer l
    (per-layer comparison from the GPU's own inputs)."""
    layers = unpack(params)
    a = f[..., None].astype(np.float64)
    acts = [a]
    for l, (W, b) in enumerate(layers):
        if acts_in is not None and acts_in[l] is not None:
            a = acts_in[l]
            acts[-1] = a
        Wl = round_bf16(W) if bf16 else W
        z = conv(a, Wl, b)
        if l < len(layers) - 1:
            a = np.maximum(z, 0.0)
            if bf16:
                a = round_bf16(a)
            acts.append(a)
        else:
            out = z[..., 0]
    return f + out, acts


def loss_and_grad(params: np.ndarray, f: np.ndarray, target: np.ndarray, bf16: bool = False):
    """Mean squared error of u_pred against target and its gradient in the parameter layout."""
    layers = unpack(params)
    u, acts = forward(params, f, bf16)
    r = u - target
    N = r.size
    loss = float(np.sum(r * r) / N)
    dz = (2.0 * r / N)[..., None]
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, b = layers[l]
        Wl = round_bf16(W) if bf16 else W
        a = acts[l]
        grads[l] = (weight_grad(a, dz), dz.sum(axis=(0, 1, 2)))
        if l > 0:
            da = conv_transpose_taps(dz, Wl)
            dz = da * (a > 0)
            if bf16:
                dz = round_bf16(dz)
    return loss, pack(grads)


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); t is the 1-based step number."""
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mhat = m / (1 - beta1 ** t)
    vhat = v / (1 - beta2 ** t)
    w = w - lr * mhat / (np.sqrt(vhat) + eps)
    return w, m, v
