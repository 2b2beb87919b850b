"""The surrogate's kernels against the FP64 reference layers, on bf16-exact
inputs and weights (so only FP32 accumulation and the final rounding of bf16
outputs remain), and the batch calls that let the lattice audit it."""
import sys

import numpy as np
import pytest

import lbsynth as ls
from oracle import conv_oracle as co

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def _bf16(torch, a):
    """bf16 device tensor of a and its exact FP64 values."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16)
    return t.cuda(), t.to(torch.float64).numpy()


def _bf16_exact_f32(torch, a):
    """FP32 values that bf16 represents exactly (weights the kernels pack)."""
    t = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float32)
    return t.numpy()


def _f64(t):
    return t.detach().cpu().double().numpy()


# (ci, co) of the kernel, (cir, cor) real channels of the layer, mode
CONV_CASES = [
    (8, 48, 6, 48, 0),    # first layer: 2 padded input channels ignored
    (48, 48, 48, 48, 1),  # residual
    (48, 16, 48, 3, 2),   # output: 3 real of 16
    (16, 48, 48, 3, 3),   # input gradient of the output layer (48 -> 3, transposed)
    (48, 48, 48, 48, 3),  # input gradient of a residual layer
]
SHAPES = [(2, 9, 80), (1, 5, 40), (1, 4, 64), (3, 1, 130), (1, 3, 1)]


def _conv_case(torch, case, shape, blocks=0, sample=None):
    """Run one layer kernel on seeded bf16-exact data and compare it with the
    FP64 reference: on every pixel, or (sample = count) on that many seeded
    pixels computed one by one."""
    from paper_1307_6703_amd import surrogate as sg
    ci, cout, cir, cor, mode = case
    B, H, W = shape
    g = _rng(hash((ci, cout, mode, B, H, W)) % 2**32)
    x_d, x = _bf16(torch, g.normal(size=(B, H, W, ci)))
    if mode == 3:
        # forward layer cir -> cor; the kernel maps its gradient (ci = padded
        # cor channels) back to cir = cout channels
        w = _bf16_exact_f32(torch, g.normal(0, 0.2, size=(3, 3, cir, cor)))
        wp = sg.pack(torch.from_numpy(w.reshape(-1)).cuda(), cir, cor, cout, ci, transposed=True)
    else:
        w = _bf16_exact_f32(torch, g.normal(0, 0.2, size=(3, 3, cir, cor)))
        wp = sg.pack(torch.from_numpy(w.reshape(-1)).cuda(), cir, cor, ci, cout)
    w64 = w.astype(np.float64)
    bias = g.normal(0, 0.1, size=cor).astype(np.float32)
    bias_d = torch.from_numpy(bias).cuda()
    b64 = bias.astype(np.float64)
    idx = None
    if sample:
        idx = np.stack([g.integers(0, B, sample), g.integers(0, H, sample),
                        g.integers(0, W, sample)], axis=1)
    at = (lambda a: a) if idx is None else (lambda a: a[idx[:, 0], idx[:, 1], idx[:, 2]])
    conv = (lambda xx, ww, bb: co.conv3x3(xx, ww, bb)) if idx is None else \
        (lambda xx, ww, bb: co.conv3x3_at(xx, ww, bb, idx))
    if mode == 0:
        y, z = sg.conv(0, ci, cout, x_d, wp, bias_d, want_z=True, blocks=blocks)
        v = conv(x[..., :cir], w64, b64)
        exp_y, exp_z = co.silu(v), v
    elif mode == 1:
        r_d, r = _bf16(torch, g.normal(size=(B, H, W, cout)))
        y, z = sg.conv(1, ci, cout, x_d, wp, bias_d, res=r_d, want_z=True, blocks=blocks)
        v = conv(x, w64, b64)
        exp_y, exp_z = at(r) + co.silu(v), v
    elif mode == 2:
        yf = sg.conv(2, ci, cout, x_d, wp, bias_d, nout=cor, blocks=blocks)
        torch.cuda.synchronize()
        exp = conv(x, w64, b64)
        got = at(_f64(yf))
        assert got.shape == exp.shape
        assert np.max(np.abs(got - exp)) <= 1e-5 * np.max(np.abs(exp))
        return
    else:
        r_d, r = _bf16(torch, g.normal(size=(B, H, W, cout)))
        zp_d, zp = _bf16(torch, g.normal(size=(B, H, W, cout)))
        y, z = sg.conv(3, ci, cout, x_d, wp, None, res=r_d, zprev=zp_d, want_z=True, blocks=blocks)
        dg = co.conv3x3_dgrad(x[..., :cor], w64) if idx is None else \
            co.conv3x3_dgrad_at(x[..., :cor], w64, idx)
        gsum = dg + at(r)
        exp_y, exp_z = gsum * co.silu_grad(at(zp)), gsum
    torch.cuda.synchronize()
    for got_t, exp in ((y, exp_y), (z, exp_z)):
        got = at(_f64(got_t))
        scale = np.max(np.abs(exp))
        # bf16 output: half an ulp of rounding (2^-9 relative) plus FP32 accumulation
        assert np.all(np.abs(got - exp) <= 2.0 ** -8 * np.abs(exp) + 1e-5 * scale), \
            np.max(np.abs(got - exp) - 2.0 ** -8 * np.abs(exp))


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_matches_reference(torch_cuda, case, shape):
    _say("conv", case, shape)
    _conv_case(torch_cuda, case, shape)


# Images of 16 tiles or more (8-row x 64-column tiles, ragged in both
# directions) on grids of 1-3 workgroups: every workgroup walks several tiles,
# so the next-tile prefetch and the reuse of the LDS tile run under the check.
@pytest.mark.parametrize("blocks", [1, 2, 3])
@pytest.mark.parametrize("shape", [(2, 17, 130), (1, 32, 256)])
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_multi_tile_walk(torch_cuda, case, shape, blocks):
    _say("conv walk", case, shape, blocks)
    _conv_case(torch_cuda, case, shape, blocks=blocks)


# Full size (8 lattices of 128 x 256, 512 tiles) in the default persistent
# grid, checked on 2048 seeded pixels computed one by one.
@pytest.mark.parametrize("case", CONV_CASES)
def test_conv_full_size_sampled(torch_cuda, case):
    _say("conv full size", case)
    _conv_case(torch_cuda, case, (8, 128, 256), sample=2048)


def test_pack_layout_is_bitwise(torch_cuda):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("pack")
    g = _rng(5)
    cir, cor, CI, CO = 6, 3, 8, 16
    w = g.normal(size=(9, cir, cor)).astype(np.float32)
    fwd = sg.pack(torch.from_numpy(w.reshape(-1)).cuda(), cir, cor, CI, CO).cpu().float().numpy()
    bwd = sg.pack(torch.from_numpy(w.reshape(-1)).cuda(), cir, cor, CI, CO, True).cpu().float().numpy()
    wb = _bf16_exact_f32(torch, w)
    kf, kb = sg.kpad(CI), sg.kpad(CO)
    ef = np.zeros((CO, kf), np.float32)
    eb = np.zeros((CI, kb), np.float32)
    for tap in range(9):
        for ci in range(cir):
            for c in range(cor):
                ef[c, tap * CI + ci] = wb[tap, ci, c]
                eb[ci, tap * CO + c] = wb[8 - tap, ci, c]
    assert np.array_equal(fwd.reshape(CO, kf), ef)
    assert np.array_equal(bwd.reshape(CI, kb), eb)


@pytest.mark.parametrize("ci,cout,cir,cor", [(8, 48, 6, 48), (48, 48, 48, 48), (48, 16, 48, 3)])
@pytest.mark.parametrize("shape,blocks", [((2, 9, 80), 512), ((1, 5, 130), 7), ((1, 3, 1), 1)])
def test_wgrad_matches_reference(torch_cuda, ci, cout, cir, cor, shape, blocks):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("wgrad", ci, cout, shape, blocks)
    B, H, W = shape
    g = _rng(ci * 1000 + cout + W)
    x_d, x = _bf16(torch, g.normal(size=(B, H, W, ci)))
    gz_d, gz = _bf16(torch, g.normal(size=(B, H, W, cout)))
    dw, db = sg.wgrad(ci, cout, cir, cor, x_d, gz_d, scale=0.5, blocks=blocks)
    torch.cuda.synchronize()
    ew, eb = co.conv3x3_wgrad(x[..., :cir], gz[..., :cor])
    for got, exp in ((_f64(dw), 0.5 * ew.reshape(-1)), (_f64(db), 0.5 * eb)):
        assert np.max(np.abs(got - exp)) <= 1e-5 * np.max(np.abs(exp)) + 1e-12


def test_bias_grad_mse_adam(torch_cuda):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("bias grad, loss, adam")
    g = _rng(9)
    gz_d, gz = _bf16(torch, g.normal(size=(3, 7, 33, 16)))
    db = _f64(sg.bias_grad(gz_d, 3, scale=0.25))
    assert np.allclose(db, 0.25 * gz.reshape(-1, 16).sum(0)[:3], rtol=1e-6, atol=1e-6)
    pred = g.normal(size=(3, 7, 33, 3)).astype(np.float32)
    tgt = g.normal(size=(3, 7, 33, 3)).astype(np.float32)
    loss, gout = sg.mse(torch.from_numpy(pred).cuda(), torch.from_numpy(tgt).cuda())
    d32 = (pred - tgt).astype(np.float32)
    assert abs(float(loss.item()) - np.mean(d32.astype(np.float64) ** 2)) <= 1e-12
    eg = torch.from_numpy(2 * d32).to(torch.bfloat16).float().numpy()
    got = gout.cpu().float().numpy()
    assert np.array_equal(got[..., :3], eg) and np.all(got[..., 3:] == 0)
    p = g.normal(size=1000).astype(np.float32)
    gr = g.normal(size=1000).astype(np.float32)
    m = np.zeros(1000, np.float32)
    v = np.zeros(1000, np.float32)
    P, G, M, V = (torch.from_numpy(a.copy()).cuda() for a in (p, gr, m, v))
    ep, em, ev = p.astype(np.float64), m.astype(np.float64), v.astype(np.float64)
    for t in (1, 2, 3):
        sg.adam(P, G, M, V, t, lr=1e-2)
        ep, em, ev = co.adam_step(ep, gr.astype(np.float64), em, ev, t, lr=1e-2)
    assert np.allclose(_f64(P), ep, rtol=1e-5, atol=1e-6)


def test_field_conversions(torch_cuda):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("fields <-> tensors")
    g = _rng(12)
    B, H, W = 3, 6, 10
    f0 = np.stack([1 + 0.3 * g.normal(size=(B, H, W)), 0.05 * g.normal(size=(B, H, W)),
                   0.05 * g.normal(size=(B, H, W))], axis=1)
    f1 = f0 + 0.01 * g.normal(size=f0.shape)
    vx = (0.004 * g.normal(size=(B, W))).astype(np.float32)
    cond = np.array([[0.05, 0.9], [0.0, 0.95], [0.08, 0.86]], np.float32)
    F0, F1 = torch.from_numpy(f0).cuda(), torch.from_numpy(f1).cuda()
    s = sg.DEFAULT_SCALES
    x = sg.fields_to_input(F0, torch.from_numpy(vx).cuda(), torch.from_numpy(cond).cuda(), True)
    xe = np.zeros((B, H, W, 8), np.float32)
    xe[..., 0] = ((f0[:, 0] - 1.0) * s[0]).astype(np.float32)
    xe[..., 1] = (f0[:, 1] * s[1]).astype(np.float32)
    xe[..., 2] = (f0[:, 2] * s[1]).astype(np.float32)
    xe[..., 3] = (vx * np.float32(s[2]))[:, None, :]
    xe[:, 0, :, 4] = -cond[:, 0:1] * np.float32(s[1])
    xe[:, -1, :, 4] = cond[:, 0:1] * np.float32(s[1])
    xe[..., 5] = ((cond[:, 1] - np.float32(0.9)) * np.float32(s[3]))[:, None, None]
    xe = torch.from_numpy(xe).to(torch.bfloat16).float().numpy()
    assert np.array_equal(x.cpu().float().numpy(), xe)
    tg = sg.make_target(F0, F1).cpu().numpy()
    d = f1 - f0
    te = np.stack([d[:, 0] * s[0], d[:, 1] * s[1], d[:, 2] * s[1]], axis=-1).astype(np.float32)
    assert np.array_equal(tg, te)
    out = torch.from_numpy(te).cuda()
    back = _f64(sg.apply_output(F0, out))
    t64 = te.astype(np.float64)
    assert np.allclose(back, f0 + np.stack([t64[..., 0] / s[0], t64[..., 1] / s[1], t64[..., 2] / s[1]], 1),
                       rtol=0, atol=1e-15)
    c = sg.compare(F1, F0).cpu().numpy()
    assert np.allclose(c[:, 0], f1[:, 0].sum((1, 2)), rtol=1e-13)
    assert np.allclose(c[:, 1], f0[:, 0].sum((1, 2)), rtol=1e-13)
    assert np.allclose(c[:, 2], (np.abs(f1[:, 0] - f0[:, 0]) / f0[:, 0]).max((1, 2)), rtol=1e-14)
    assert np.all(c[:, 3] == 0)
    assert np.allclose(c[:, 4], ((f1[:, 0] - f0[:, 0]) ** 2).sum((1, 2)), rtol=1e-13)
    assert np.allclose(c[:, 5], (f0[:, 0] ** 2).sum((1, 2)), rtol=1e-13)
    mask = torch.tensor([1, 0, 1], dtype=torch.int32).cuda()
    sg.project_mass(F1, F0, mask)
    p = _f64(F1)
    assert np.allclose(p[[0, 2], 0].sum((1, 2)), f0[[0, 2], 0].sum((1, 2)), rtol=1e-14)
    assert np.array_equal(p[1], f1[1])
    assert np.allclose(p[[0, 2], 0] - f1[[0, 2], 0],
                       ((f0[[0, 2], 0] - f1[[0, 2], 0]).sum((1, 2)) / (H * W))[:, None, None], atol=1e-14)


def _bf16_params(torch, g):
    from paper_1307_6703_amd import surrogate as sg
    parts = []
    for ci, c in sg.layer_shapes():
        parts.append(g.normal(0, 1.0 / np.sqrt(9 * ci), size=9 * ci * c))
        parts.append(g.normal(0, 0.1, size=c))
    return _bf16_exact_f32(torch, np.concatenate(parts))


def test_network_forward_and_gradients(torch_cuda):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("network forward/backward")
    g = _rng(21)
    B, H, W = 2, 12, 72
    p = _bf16_params(torch, g)
    net = sg.Net(B, H, W, train=True)
    net.set_params(p)
    x_d, x = _bf16(torch, g.normal(size=(B, H, W, 8)))
    tgt = g.normal(size=(B, H, W, 3)).astype(np.float32)
    params = sg.split_params(p)
    out_ref, cache = co.forward(params, x[..., :6])
    out = _f64(net.forward(x_d))
    # bf16 activations between the layers: a few parts in 1e3
    assert np.max(np.abs(out - out_ref)) <= 2e-2 * np.max(np.abs(out_ref))
    loss = float(net.train_step(x_d, torch.from_numpy(tgt).cuda(), 1e-3).item())
    loss_ref, gout = co.mse(out_ref, tgt.astype(np.float64))
    assert abs(loss - loss_ref) <= 1e-2 * loss_ref
    grads = _f64(net.grads())
    ref = co.backward(params, cache, gout)
    o = 0
    for (gw, gb) in ref:
        for r in (gw.reshape(-1), gb):
            gg = grads[o:o + r.size]
            o += r.size
            assert np.linalg.norm(gg - r) <= 5e-2 * np.linalg.norm(r), (o, np.linalg.norm(gg - r) / np.linalg.norm(r))
    assert o == grads.size
    # the Adam step used these gradients
    p1 = _f64(net.params())
    e1, _, _ = co.adam_step(p.astype(np.float64), grads, np.zeros_like(grads), np.zeros_like(grads), 1,
                            lr=1e-3)
    assert np.allclose(p1, e1, rtol=1e-5, atol=1e-7)
    net.close()


def test_network_forward_full_size_sampled(torch_cuda):
    # 8 lattices of 128 x 256 (the evaluation's image size) in the default
    # launch; 512 seeded pixels against the FP64 network run on each pixel's
    # receptive field only
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("network forward full size")
    g = _rng(22)
    B, H, W = 8, 128, 256
    p = _bf16_params(torch, g)
    net = sg.Net(B, H, W, train=False)
    net.set_params(p)
    x_d, x = _bf16(torch, g.normal(size=(B, H, W, 8)))
    out = _f64(net.forward(x_d))
    idx = np.stack([g.integers(0, B, 512), g.integers(0, H, 512), g.integers(0, W, 512)], axis=1)
    # rows next to the walls are among them
    idx[:8, 1] = [0, 1, 2, H - 1, H - 2, H - 3, 0, H - 1]
    exp = co.forward_at(sg.split_params(p), x[..., :6], idx)
    got = out[idx[:, 0], idx[:, 1], idx[:, 2]]
    # bf16 activations between the layers: a few parts in 1e3
    assert np.max(np.abs(got - exp)) <= 2e-2 * np.max(np.abs(exp))
    assert np.linalg.norm(got - exp) <= 1e-2 * np.linalg.norm(exp)
    net.close()


def _layer_chain(torch, sg, p_dev, x_d):
    # the network as six single-layer launches (lbs_conv), weights packed
    # from the flat parameters the way the network packs them
    outs, o = [], 0
    shapes = sg.layer_shapes()
    h = x_d
    for l, (cir, cor) in enumerate(shapes):
        CI = sg.IN_CHANNELS if l == 0 else sg.WIDTH
        CO = sg.OUT_CHANNELS if l == len(shapes) - 1 else sg.WIDTH
        w = p_dev[o:o + 9 * cir * cor]
        o += 9 * cir * cor
        b = p_dev[o:o + cor].contiguous()
        o += cor
        wp = sg.pack(w.contiguous(), cir, cor, CI, CO)
        if l == 0:
            h, _ = sg.conv(sg.FWD_FIRST, CI, CO, h, wp, bias=b)
        elif l < len(shapes) - 1:
            h, _ = sg.conv(sg.FWD_RES, CI, CO, h, wp, bias=b, res=h)
        else:
            outs = sg.conv(sg.FWD_OUT, CI, CO, h, wp, bias=b, nout=sg.OUT)
    return outs


@pytest.mark.parametrize("shape,train", [((2, 12, 64), False), ((3, 9, 128), False), ((1, 1, 64), False),
                                         ((2, 3, 192), True), ((4, 128, 256), False), ((2, 10, 72), False)])
def test_fused_residual_stack_equals_layer_chain(torch_cuda, shape, train):
    # The forward runs the four residual layers as one pass with the
    # activations kept on chip when W is a multiple of 64 (one strip: the
    # periodic halo wraps onto the strip itself; one row: both neighbours are
    # wall padding); the same products in the same order as the single-layer
    # kernel, so the output is the same bits. W = 72 takes the per-layer path.
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    B, H, W = shape
    _say("fused residual stack vs layer chain", shape, train)
    g = _rng(31)
    p = _bf16_params(torch, g)
    net = sg.Net(B, H, W, train=train)
    net.set_params(p)
    x_d, _ = _bf16(torch, g.normal(size=(B, H, W, 8)))
    out = net.forward(x_d)
    ref = _layer_chain(torch, sg, torch.from_numpy(np.asarray(p, dtype=np.float32)).cuda(), x_d)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), float((out - ref).abs().max())
    net.close()


def _draws(count, Lx, Ly, seed):
    return ls.surrogate_draws(count, seed=seed, Lx=Lx, Ly=Ly)


def test_batch_device_moments_reentry_and_subset(torch_cuda):
    from paper_1307_6703_amd import Batch
    from paper_1307_6703_amd.surrogate import _batch_for
    torch = torch_cuda
    _say("batch moments_device / set_equilibrium / step_subset")
    draws = _draws(3, 70, 20, 4)
    a = _batch_for(draws, check_every=0, drift=False)
    f0 = a.moments_device()
    torch.cuda.synchronize()
    for i in range(3):
        n, ux, uy = a.moments(i)
        assert np.array_equal(_f64(f0[i, 0]), n) and np.array_equal(_f64(f0[i, 1]), ux)
    # subset steps: instance 1 untouched, 0 and 2 as a full batch run
    with pytest.raises(Exception):
        a.step_subset(3, [1, 0, 1])
    a.step_subset(6, [1, 0, 1])
    b = _batch_for(draws, check_every=0, drift=False)
    b.step(6)
    for i in (0, 2):
        for u, v in zip(a.moments(i), b.moments(i)):
            assert np.array_equal(u, v)
    for u, v in zip(a.moments(1), (_f64(f0[1, k]) for k in range(3))):
        assert np.array_equal(u, v)
    # re-entry at the initial fields reproduces the initial state exactly
    a.set_equilibrium(f0, [1, 1, 1])
    a.step(8)
    c = _batch_for(draws, check_every=0, drift=False)
    c.step(8)
    for i in range(3):
        for u, v in zip(a.moments(i), c.moments(i)):
            assert np.array_equal(u, v)
    for bb in (a, b, c):
        bb.close()


def test_training_reduces_the_loss(torch_cuda):
    from paper_1307_6703_amd import surrogate as sg
    torch = torch_cuda
    _say("training on lattice data")
    draws = _draws(8, 64, 32, 7)
    x, tgt, status = sg.generate_data(draws, warmup=100, chunks=4, K=10)
    assert all(s == 0 for s in status)
    net = sg.Net(8, 32, 64, train=True)
    net.set_params(sg.init_params(3))
    hist = sg.train(net, x, tgt, iters=300, batch=8, lr=3e-3, log_every=50)
    first = hist[0][1]
    last = min(l for _, l in hist[-2:])
    assert np.isfinite(last) and last < 0.7 * first, hist
    net.close()


def test_audited_run_all_audits_equals_lattice(torch_cuda):
    """Every instance audited every chunk: nothing is taken from the network
    and the run is the lattice's own, bitwise."""
    from paper_1307_6703_amd import surrogate as sg
    _say("audited run, all audits")
    draws = _draws(4, 64, 32, 8)
    net = sg.Net(4, 32, 64)
    net.set_params(sg.init_params(1))
    a = sg._batch_for(draws, check_every=0, drift=False)
    run = sg.SurrogateRun(net, a, draws, K=10, audit_every=1, mass_tol=1.0)
    for _ in range(3):
        run.chunk()
    assert run.stats.fallback_rate == 1.0 and run.stats.audits == 12
    b = sg._batch_for(draws, check_every=0, drift=False)
    b.step(30)
    for i in range(4):
        for u, v in zip(a.moments(i), b.moments(i)):
            assert np.array_equal(u, v)
    for bb in (a, b):
        bb.close()
    net.close()


def test_audited_run_trust_rotation_and_mass(torch_cuda):
    """With a network that predicts no change, every audit within a loose
    tolerance passes: instances are audited on the lattice while on
    probation, then half of them per chunk (rotation), the rest re-enter
    from the prediction, and each instance keeps its FP64 mass."""
    from paper_1307_6703_amd import surrogate as sg
    _say("audited run, trust rotation and mass")
    draws = _draws(4, 64, 32, 9)
    net = sg.Net(4, 32, 64)
    net.set_params(np.zeros(sg.param_count(), np.float32))
    a = sg._batch_for(draws, check_every=0, drift=False)
    m0 = [a.reduce(i)["mass"] for i in range(4)]
    run = sg.SurrogateRun(net, a, draws, K=10, tol=1.0, audit_every=2)
    accepted = [run.chunk() for _ in range(4)]
    st = run.stats
    assert [list(np.nonzero(x)[0]) for x in accepted] == [[], [0, 2], [1, 3], [0, 2]]
    assert (st.audits, st.audit_failures, st.surrogate_chunks, st.lattice_chunks) == (10, 0, 6, 10)
    for i in range(4):
        m = a.reduce(i)["mass"]
        assert abs(m - m0[i]) <= 1e-6 * m0[i]
    a.close()
    net.close()


def test_audited_run_rejects_beyond_tolerance(torch_cuda):
    """A zero tolerance fails every audit: nothing leaves probation and the
    run stays on the lattice."""
    from paper_1307_6703_amd import surrogate as sg
    _say("audited run, rejection")
    draws = _draws(4, 64, 32, 10)
    net = sg.Net(4, 32, 64)
    net.set_params(sg.init_params(2))
    a = sg._batch_for(draws, check_every=0, drift=False)
    run = sg.SurrogateRun(net, a, draws, K=10, tol=0.0, audit_every=2, mass_tol=1.0)
    for _ in range(4):
        run.chunk()
    st = run.stats
    assert (st.audits, st.audit_failures, st.surrogate_chunks, st.lattice_chunks) == (16, 16, 0, 16)
    a.close()
    net.close()


def test_persistence_baseline_equals_zero_network(torch_cuda):
    """The persistence baseline (no network) runs exactly as a network whose
    output is zero: same accepted instances, statistics and final state."""
    from paper_1307_6703_amd import surrogate as sg
    _say("audited run, persistence baseline")
    draws = _draws(4, 64, 32, 11)
    net = sg.Net(4, 32, 64)
    net.set_params(np.zeros(sg.param_count(), np.float32))
    a = sg._batch_for(draws, check_every=0, drift=False)
    b = sg._batch_for(draws, check_every=0, drift=False)
    ra = sg.SurrogateRun(net, a, draws, K=10, tol=0.05, audit_every=2)
    rb = sg.SurrogateRun(None, b, draws, K=10, tol=0.05, audit_every=2, predictor="persist")
    for _ in range(5):
        assert np.array_equal(ra.chunk(), rb.chunk())
    assert ra.stats == rb.stats
    for i in range(4):
        for u, v in zip(a.moments(i), b.moments(i)):
            assert np.array_equal(u, v)
    with pytest.raises(ValueError):
        sg.SurrogateRun(None, a, draws, K=10)
    for bb in (a, b):
        bb.close()
    net.close()


def test_shift_reentry_keeps_the_non_equilibrium_part(torch_cuda):
    """lb_batch_shift_equilibrium_device: at equal fields the populations stay
    the same bits; from an equilibrium state it agrees with replacing the
    populations by f_eq (up to FP32 rounding); the mass moves by the change
    of the density field; a shift there and back returns the state."""
    from paper_1307_6703_amd.surrogate import _batch_for
    torch = torch_cuda
    _say("shift re-entry")
    draws = _draws(3, 70, 20, 12)
    a, b, c = (_batch_for(draws, check_every=0, drift=False) for _ in range(3))
    for bb in (a, b, c):
        bb.step(40)  # a state with a non-equilibrium part
    f0 = a.moments_device()
    yy, xx = torch.meshgrid(torch.arange(20, device="cuda"), torch.arange(70, device="cuda"),
                            indexing="ij")
    f1 = f0.clone()
    f1[:, 0] *= 1.0 + 0.01 * torch.sin(2 * np.pi * xx / 70).double()
    f1[:, 1] += 0.002 * torch.cos(2 * np.pi * yy / 20).double()
    m0 = [a.reduce(i)["mass"] for i in range(3)]
    # equal fields: bit for bit the run without re-entry
    a.shift_equilibrium(f0, f0, [1, 1, 1])
    a.step(10)
    c.step(10)
    for i in range(3):
        for u, v in zip(a.moments(i), c.moments(i)):
            assert np.array_equal(u, v)
    # there and back: the state returns up to FP32 rounding
    b.shift_equilibrium(f0, f1, [1, 0, 1])
    for i in (0, 2):
        n, ux, _ = b.moments(i)
        assert np.array_equal(n, _f64(f1[i, 0])) and np.array_equal(ux, _f64(f1[i, 1]))
        dm = float((f1[i, 0] - f0[i, 0]).sum())
        assert abs(b.reduce(i)["mass"] - (m0[i] + dm)) <= 1e-6 * m0[i]
    assert np.array_equal(b.moments(1)[0], _f64(f0[1, 0]))
    b.shift_equilibrium(f1, f0, [1, 0, 1])
    b.step(10)
    for i in range(3):
        for u, v in zip(b.moments(i), c.moments(i)):
            assert np.allclose(u, v, rtol=0, atol=1e-5)
    # from an equilibrium state (just initialised) shift == replace
    e, g = (_batch_for(draws, check_every=0, drift=False) for _ in range(2))
    fi = e.moments_device()
    fj = fi.clone()
    fj[:, 0] *= 1.0 + 0.01 * torch.sin(2 * np.pi * xx / 70).double()
    e.set_equilibrium(fj, [1, 1, 1])
    g.shift_equilibrium(fi, fj, [1, 1, 1])
    e.step(10)
    g.step(10)
    for i in range(3):
        for u, v in zip(e.moments(i), g.moments(i)):
            assert np.allclose(u, v, rtol=0, atol=1e-5)
    # errors: no "from" fields, a batch of uneven sizes
    import ctypes
    from paper_1307_6703_amd import Batch, LBError, lbvdw
    m = np.ones(3, np.int32)
    st = lbvdw.load_library().lb_batch_shift_equilibrium_device(
        a._h, None, ctypes.c_void_p(f1.data_ptr()), m.ctypes.data_as(lbvdw._I32P))
    assert st == lbvdw.LB_EINVAL
    un = Batch([dict(Lx=70, Ly=20), dict(Lx=64, Ly=20)], fp32=True)
    un.init(0, np.ones((20, 70)))
    un.init(1, np.ones((20, 64)))
    with pytest.raises(LBError):
        un.shift_equilibrium(f1[:2], f1[:2], [1, 1])
    for bb in (a, b, c, e, g, un):
        bb.close()


def test_budget_policy_spaces_the_audits(torch_cuda):
    """Audits spaced by a run-level error budget: with budget 0 every chunk
    after the probation audit is audited again (once the first audit has
    measured a nonzero error); with a budget no chunk can exhaust, a trusted
    instance is audited only after the longest gap; the results agree with
    the rotation policy's bookkeeping."""
    from paper_1307_6703_amd import surrogate as sg
    _say("audited run, budget policy")
    draws = _draws(4, 64, 32, 13)
    net = sg.Net(4, 32, 64)
    net.set_params(np.zeros(sg.param_count(), np.float32))
    a = sg._batch_for(draws, check_every=0, drift=False)
    run = sg.SurrogateRun(net, a, draws, K=10, tol=1.0, audit_every=100, budget=0.0)
    acc = [run.chunk() for _ in range(4)]
    assert all(not x.any() for x in acc)  # every chunk on the lattice
    assert run.stats.audits == 16 and run.stats.audit_failures == 0
    assert (run.est > 0).all()
    b = sg._batch_for(draws, check_every=0, drift=False)
    run = sg.SurrogateRun(net, b, draws, K=10, tol=1.0, audit_every=3, budget=1e9)
    acc = [list(np.nonzero(run.chunk())[0]) for _ in range(7)]
    # probation audit, two trusted chunks, audit at the gap, two more, audit
    assert acc == [[], [0, 1, 2, 3], [0, 1, 2, 3], [], [0, 1, 2, 3], [0, 1, 2, 3], []]
    assert run.stats.audits == 12 and run.stats.surrogate_chunks == 16
    with pytest.raises(ValueError):
        sg.SurrogateRun(net, b, draws, K=10, budget=-1.0)
    for bb in (a, b):
        bb.close()
    net.close()


def test_experiment_runs_end_to_end(torch_cuda):
    """The benchmark's surrogate experiment at a toy size: data, training,
    every evaluation variant, and the lattice-only control matching the
    reference run."""
    from paper_1307_6703_amd import surrogate as sg
    _say("surrogate experiment, toy size")
    out = sg.experiment(H=32, W=64, train_count=8, test_count=8, train_windows=((20, 2), (60, 2)),
                        eval_starts=(20,), K=10, iters=40, batch=4, train_seconds=10.0,
                        eval_chunks=3, audit_every=2)
    assert out["train"]["iterations"] == 40 and out["train_samples"] > 0
    win = out["eval"]["windows"][0]
    for key in ("lattice_control", "audit_max", "persist_max",
                "persist_max_eq_reentry", "audit_max_budget", "persist_max_budget"):
        v = win[key]
        # FP32 storage; subset steps skip the drift shift: the bar is the
        # run's mass tolerance (1e-4), with margin
        assert v["speedup"] > 0 and v["diverged"] == 0 and v["mass_drift_max"] < 1e-6, key
    assert win["lattice_control"]["fallback_rate"] == 1.0
    assert win["lattice_control"]["final_frac_within_tol"] == 1.0
    assert out["forward"]["ms"] > 0


def test_trained_network_beats_persistence(torch_cuda):
    """What the network adds, at a small size: trained on lattice chunks
    while the phases separate (fields moving fast), it predicts the change
    over a chunk better than the prediction that nothing changes, both on
    its training windows and in the audits against the lattice on other
    draws."""
    from paper_1307_6703_amd import surrogate as sg
    _say("trained network vs persistence")
    out = sg.experiment(H=32, W=64, train_count=24, test_count=8, train_windows=((20, 6), (60, 6)),
                        eval_starts=(20,), K=10, iters=1500, batch=8, lr=2e-3, train_seconds=60.0,
                        eval_chunks=4, audit_every=1)
    tr = out["train"]
    _say("loss per window", tr["dataset_loss_after_per_window"], "persistence",
         tr["persistence_loss_per_window"])
    for net_l, per_l in zip(tr["dataset_loss_after_per_window"], tr["persistence_loss_per_window"]):
        assert net_l < 0.5 * per_l
    win = out["eval"]["windows"][0]
    e_net = win["audit_max"]["audit_error_median"]
    e_per = win["persist_max"]["audit_error_median"]
    _say("audit error median: network", e_net, "persistence", e_per)
    assert e_net < 0.5 * e_per
