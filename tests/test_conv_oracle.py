"""Pins of the surrogate's FP64 reference layers: brute-force loops on tiny
tensors, finite-difference gradients, closed forms."""
import numpy as np
import pytest

from oracle import conv_oracle as co


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _brute_conv(x, w, b):
    B, H, W, Ci = x.shape
    Co = w.shape[3]
    y = np.zeros((B, H, W, Co))
    for n in range(B):
        for h in range(H):
            for xx in range(W):
                for c in range(Co):
                    acc = b[c]
                    for dy in (-1, 0, 1):
                        hh = h + dy
                        if hh < 0 or hh >= H:
                            continue
                        for dx in (-1, 0, 1):
                            for ci in range(Ci):
                                acc += x[n, hh, (xx + dx) % W, ci] * w[dy + 1, dx + 1, ci, c]
                    y[n, h, xx, c] = acc
    return y


def test_conv_matches_brute_force_loops():
    g = _rng(1)
    x = g.normal(size=(2, 4, 5, 3))
    w = g.normal(size=(3, 3, 3, 2))
    b = g.normal(size=2)
    assert np.allclose(co.conv3x3(x, w, b), _brute_conv(x, w, b), atol=1e-12)


def test_delta_kernel_shifts():
    # a single tap at (dy, dx) = (0, +1) reads the right neighbour (wrapped)
    g = _rng(2)
    x = g.normal(size=(1, 3, 6, 1))
    w = np.zeros((3, 3, 1, 1))
    w[1, 2, 0, 0] = 1.0
    assert np.allclose(co.conv3x3(x, w)[0, :, :, 0], np.roll(x[0, :, :, 0], -1, axis=1))
    # (dy, dx) = (+1, 0) reads the row above; the top row sees zero padding
    w = np.zeros((3, 3, 1, 1))
    w[2, 1, 0, 0] = 1.0
    y = co.conv3x3(x, w)[0, :, :, 0]
    assert np.allclose(y[:-1], x[0, 1:, :, 0]) and np.allclose(y[-1], 0.0)


def _num_grad(f, a, eps=1e-6):
    g = np.zeros_like(a)
    it = np.nditer(a, flags=["multi_index"])
    for _ in it:
        i = it.multi_index
        old = a[i]
        a[i] = old + eps
        fp = f()
        a[i] = old - eps
        fm = f()
        a[i] = old
        g[i] = (fp - fm) / (2 * eps)
    return g


def test_conv_gradients_match_finite_differences():
    g = _rng(3)
    x = g.normal(size=(2, 4, 5, 3))
    w = g.normal(size=(3, 3, 3, 2))
    b = g.normal(size=2)
    c = g.normal(size=(2, 4, 5, 2))  # loss = sum(c * y)
    loss = lambda: float((c * co.conv3x3(x, w, b)).sum())
    assert np.allclose(co.conv3x3_dgrad(c, w), _num_grad(loss, x), atol=1e-6)
    gw, gb = co.conv3x3_wgrad(x, c)
    assert np.allclose(gw, _num_grad(loss, w), atol=1e-6)
    assert np.allclose(gb, _num_grad(loss, b), atol=1e-6)


def test_network_gradients_match_finite_differences():
    g = _rng(4)
    chans = [3, 6, 6, 6, 2]
    params = [(0.3 * g.normal(size=(3, 3, a, bb)), 0.1 * g.normal(size=bb))
              for a, bb in zip(chans[:-1], chans[1:])]
    x = g.normal(size=(1, 4, 5, 3))
    t = g.normal(size=(1, 4, 5, 2))

    def loss():
        return co.mse(co.forward(params, x)[0], t)[0]

    out, cache = co.forward(params, x)
    _, gout = co.mse(out, t)
    grads = co.backward(params, cache, gout)
    for (w, b), (gw, gb) in zip(params, grads):
        assert np.allclose(gw, _num_grad(loss, w), atol=1e-7, rtol=1e-5)
        assert np.allclose(gb, _num_grad(loss, b), atol=1e-7, rtol=1e-5)


def test_silu_derivative():
    z = np.linspace(-6, 6, 101)
    h = 1e-6
    assert np.allclose(co.silu_grad(z), (co.silu(z + h) - co.silu(z - h)) / (2 * h), atol=1e-8)


def test_first_adam_step_moves_by_lr_times_sign():
    # with bias correction, the first step is lr * g / (|g| + eps)
    g = np.array([0.3, -2.0, 1e-3])
    p, m, v = co.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def _idx(g, B, H, W, P):
    return np.stack([g.integers(0, B, P), g.integers(0, H, P), g.integers(0, W, P)], axis=1)


def test_pointwise_conv_matches_brute_force():
    # the pointwise forms used for full-size checks, against the loops above
    g = _rng(31)
    x = g.normal(size=(2, 5, 6, 3))
    w = g.normal(size=(3, 3, 3, 4))
    b = g.normal(size=4)
    full = _brute_conv(x, w, b)
    idx = np.array([[n, h, c] for n in range(2) for h in range(5) for c in range(6)])
    assert np.allclose(co.conv3x3_at(x, w, b, idx), full[idx[:, 0], idx[:, 1], idx[:, 2]],
                       atol=1e-12)
    # the input gradient of a conv is the conv with flipped, transposed taps
    wt = np.transpose(w[::-1, ::-1], (0, 1, 3, 2))
    gy = g.normal(size=(2, 5, 6, 4))
    full_dg = _brute_conv(gy, wt, np.zeros(3))
    assert np.allclose(co.conv3x3_dgrad_at(gy, w, idx), full_dg[idx[:, 0], idx[:, 1], idx[:, 2]],
                       atol=1e-12)


def test_pointwise_forward_matches_whole_image():
    # every pixel, including the wall rows and wrapped columns, of a network
    # deeper than the image is tall
    g = _rng(32)
    params = [(g.normal(0, 0.3, size=(3, 3, 4, 5)), g.normal(0, 0.1, size=5)),
              (g.normal(0, 0.3, size=(3, 3, 5, 5)), g.normal(0, 0.1, size=5)),
              (g.normal(0, 0.3, size=(3, 3, 5, 5)), g.normal(0, 0.1, size=5)),
              (g.normal(0, 0.3, size=(3, 3, 5, 2)), g.normal(0, 0.1, size=2))]
    x = g.normal(size=(2, 3, 7, 4))
    out, _ = co.forward(params, x)
    idx = np.array([[n, h, c] for n in range(2) for h in range(3) for c in range(7)])
    got = co.forward_at(params, x, idx)
    assert np.allclose(got, out[idx[:, 0], idx[:, 1], idx[:, 2]], atol=1e-12)
