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


def _patches(x, idx, r):
    """Patches of x of radius r around the pixels idx (rows (n, h, w)):
    [P, 2r + 1, 2r + 1, C], columns wrapped, rows outside the image zero;
    also the mask [P, 2r + 1] of patch rows inside the image."""
    B, H, W, C = x.shape
    n, h, w = idx[:, 0], idx[:, 1], idx[:, 2]
    off = np.arange(-r, r + 1)
    rows = h[:, None] + off[None, :]
    cols = (w[:, None] + off[None, :]) % W
    inside = (rows >= 0) & (rows < H)
    rc = np.clip(rows, 0, H - 1)
    p = x[n[:, None, None], rc[:, :, None], cols[:, None, :]]
    return p * inside[:, :, None, None], inside


def conv3x3_at(x, w, b, idx):
    """conv3x3(x, w, b) at the pixels idx only ([P, 3] rows (n, h, w)):
    [P, C_out], from the 3x3 neighbourhood of each pixel."""
    p, _ = _patches(x, idx, 1)
    y = np.einsum("pijc,ijcd->pd", p, w)
    return y + b if b is not None else y


def conv3x3_dgrad_at(gy, w, idx):
    """conv3x3_dgrad(gy, w) at the pixels idx only: [P, C_in]."""
    p, _ = _patches(gy, idx, 1)
    # gx[h, x] = sum gy[h - dy, x - dx] w[dy + 1, dx + 1]: the flipped patch
    return np.einsum("pijd,ijcd->pc", p[:, ::-1, ::-1], w)


def forward_at(params, x, idx):
    """forward(params, x)[0] at the pixels idx only: [P, C_out]. Each pixel's
    output depends on the input within len(params) pixels; the network runs
    on that patch, with the rows outside the image held at zero before every
    layer (the zero padding of each convolution) and the columns wrapped."""
    L = len(params)
    h, inside = _patches(x, idx, L)
    mask = inside[:, :, None, None].astype(h.dtype)  # rows only; broadcast over columns
    for li, (w, b) in enumerate(params):
        # a valid 3x3 convolution over the patch: it shrinks by one pixel per side
        P, S = h.shape[0], h.shape[1]
        z = np.zeros((P, S - 2, S - 2, w.shape[3]))
        for dy in range(3):
            for dx in range(3):
                z += np.tensordot(h[:, dy:S - 2 + dy, dx:S - 2 + dx], w[dy, dx], axes=([3], [0]))
        z += b
        mask = mask[:, 1:-1]
        if li == 0:
            h = silu(z) * mask
        elif li < L - 1:
            h = (h[:, 1:-1, 1:-1] + silu(z)) * mask
        else:
            return z[:, 0, 0]
    raise ValueError("network needs at least one layer")


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
