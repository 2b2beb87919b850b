"""FP64 reference of the learned surrogate's layers (test infrastructure only).

The surrogate is not part of the paper: it is a small residual convolutional
network that advances the lattice's (n, u) fields K steps at a time. This
module is its plain CPU definition, used to check the HIP kernels. Tensors
are NHWC: [batch, rows (y), columns (x), channels]. A 3x3 convolution wraps
around in x (the lattice is periodic along the flow) and pads y with zeros
(walls). Weights are [3, 3, C_in, C_out] indexed [dy + 1, dx + 1, ci, co].

Only tests/ and the CPU-baseline leg of bench.py use this module.
"""
from __future__ import annotations

import numpy as np


def _shifted(x, dy, dx):
    """x at (h + dy, w + dx): zero outside the rows, wrapped in columns."""
    B, H, W, C = x.shape
    out = np.zeros_like(x)
    src = np.roll(x, -dx, axis=2)
    if dy >= 0:
        out[:, :H - dy] = src[:, dy:]
    else:
        out[:, -dy:] = src[:, :H + dy]
    return out


def conv3x3(x, w, b=None):
    """y[n,h,x,co] = b[co] + sum_{dy,dx,ci} x[n,h+dy,x+dx,ci] w[dy+1,dx+1,ci,co]."""
    B, H, W, _ = x.shape
    y = np.zeros((B, H, W, w.shape[3]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            y += np.tensordot(_shifted(x, dy, dx), w[dy + 1, dx + 1], axes=([3], [0]))
    if b is not None:
        y += b
    return y


def conv3x3_dgrad(gy, w):
    """Gradient of conv3x3 with respect to its input: the transposed
    convolution sum_{dy,dx,co} gy[n,h-dy,x-dx,co] w[dy+1,dx+1,ci,co]."""
    B, H, W, _ = gy.shape
    gx = np.zeros((B, H, W, w.shape[2]))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            gx += np.tensordot(_shifted(gy, -dy, -dx), w[dy + 1, dx + 1], axes=([3], [1]))
    return gx


def conv3x3_wgrad(x, gy):
    """Gradients of conv3x3 with respect to weights and bias."""
    Ci, Co = x.shape[3], gy.shape[3]
    gw = np.zeros((3, 3, Ci, Co))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            xs = _shifted(x, dy, dx)
            gw[dy + 1, dx + 1] = np.tensordot(xs, gy, axes=([0, 1, 2], [0, 1, 2]))
    return gw, gy.sum(axis=(0, 1, 2))


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(params, x):
    """Network: h1 = silu(conv(x)); h_{k+1} = h_k + silu(conv(h_k)) for the
    residual layers; out = conv(h_last). Returns (out, cache)."""
    cache = {"x": x, "z": [], "h": [x]}
    h = x
    L = len(params)
    for li, (w, b) in enumerate(params):
        z = conv3x3(h, w, b)
        if li == 0:
            h = silu(z)
        elif li < L - 1:
            h = h + silu(z)
        else:
            cache["z"].append(z)
            return z, cache
        cache["z"].append(z)
        cache["h"].append(h)
    raise ValueError("network needs at least one layer")


def backward(params, cache, gout):
    """Gradients of a scalar loss with respect to every (w, b), given
    d loss / d out."""
    L = len(params)
    grads = [None] * L
    g = gout
    for li in range(L - 1, -1, -1):
        w, _ = params[li]
        hin = cache["h"][li]
        if li == L - 1:
            gz = g
        else:
            gz = g * silu_grad(cache["z"][li])
        gw, gb = conv3x3_wgrad(hin, gz)
        grads[li] = (gw, gb)
        gin = conv3x3_dgrad(gz, w)
        if 0 < li < L - 1:
            gin = gin + g  # residual path
        g = gin
    return grads


def mse(pred, target):
    """Mean squared error over all elements and its gradient."""
    d = pred - target
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam_step(p, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), t counted from 1. Returns new p, m, v."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
