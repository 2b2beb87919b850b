"""lbs_wgrad_noalloc (static device scratch, no allocation) against lbs_wgrad
(caller scratch): the same kernels on the same inputs, so the weight and
bias gradients must be the same bits. Two calls in a row, the second on a
smaller input, so the scratch left by the first call cannot leak into the
second; sizes beyond the static scratch are rejected before any launch."""
import ctypes
import sys

import numpy as np
import pytest

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


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _inputs(torch, g, B, H, W, ci, co):
    x = torch.from_numpy(g.normal(size=(B, H, W, ci)).astype(np.float32)).to(torch.bfloat16).cuda()
    gz = torch.from_numpy(g.normal(size=(B, H, W, co)).astype(np.float32)).to(torch.bfloat16).cuda()
    return x, gz


def _both(torch, lib, ci, co, cir, cor, x, gz, blocks, scale):
    from paper_1307_6703_amd import surrogate as sg
    B, H, W, _ = x.shape
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    dw_ref, db_ref = sg.wgrad(ci, co, cir, cor, x, gz, scale=scale, blocks=blocks)
    dw = torch.full((9 * cir * cor,), float("nan"), dtype=torch.float32, device="cuda")
    db = torch.full((cor,), float("nan"), dtype=torch.float32, device="cuda")
    st = lib.lbs_wgrad_noalloc(ci, co, cir, cor, _vp(x), _vp(gz), B, H, W, ctypes.c_float(scale),
                               blocks, _vp(dw), _vp(db), stream)
    assert st == 0, lib.lb_last_error().decode()
    torch.cuda.synchronize()
    return dw.cpu().numpy(), db.cpu().numpy(), dw_ref.cpu().numpy(), db_ref.cpu().numpy()


@pytest.mark.parametrize("ci,co,cir,cor,blocks", [(48, 48, 48, 48, 160), (8, 48, 6, 48, 512),
                                                   (48, 16, 48, 3, 37)])
def test_noalloc_wgrad_equals_workspace_wgrad(torch_cuda, ci, co, cir, cor, blocks):
    from paper_1307_6703_amd import load_library
    torch = torch_cuda
    lib = load_library()
    g = np.random.Generator(np.random.PCG64(ci * 1000 + cor))
    # a large call, then a smaller one (fewer pixels: fewer work units, so a
    # smaller grid whose reduction must not read the first call's partials)
    for (B, H, W) in ((4, 64, 256), (1, 9, 70)):
        _say("wgrad noalloc", ci, co, cir, cor, blocks, (B, H, W))
        x, gz = _inputs(torch, g, B, H, W, ci, co)
        dw, db, dw_ref, db_ref = _both(torch, lib, ci, co, cir, cor, x, gz, blocks, 1.0 / (B * H * W))
        assert np.all(np.isfinite(dw)) and np.all(np.isfinite(db))
        assert np.array_equal(dw, dw_ref) and np.array_equal(db, db_ref)


def test_noalloc_wgrad_rejects_oversized_scratch(torch_cuda):
    from paper_1307_6703_amd import load_library
    torch = torch_cuda
    lib = load_library()
    _say("wgrad noalloc limit")
    x, gz = _inputs(torch, np.random.Generator(np.random.PCG64(3)), 1, 8, 64, 48, 48)
    dw = torch.zeros(9 * 48 * 48, dtype=torch.float32, device="cuda")
    db = torch.zeros(48, dtype=torch.float32, device="cuda")
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    st = lib.lbs_wgrad_noalloc(48, 48, 48, 48, _vp(x), _vp(gz), 1, 8, 64, ctypes.c_float(1.0), 170,
                               _vp(dw), _vp(db), stream)
    assert st == -1 and "static scratch" in lib.lb_last_error().decode()
    torch.cuda.synchronize()
    assert float(dw.abs().sum()) == 0.0  # nothing ran
