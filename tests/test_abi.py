"""The C ABI on the CPU: the library loads, exports every symbol the header
declares, and rejects bad parameters before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1307_6703_amd import lbvdw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", h) for h in ("lbvdw.h", "lbd2q17.h", "lbsurrogate.h")]


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(?:lb_status|const char\*)\s+(lb(?:s|17)?_\w+)\s*\(", src))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lbvdw.LIB_PATH):
        from paper_1307_6703_amd import build
        build.build()
    return lbvdw.load_library()


def test_header_declares_the_documented_calls():
    names = _declared()
    for must in ("lb_create", "lb_init_lattice", "lb_step_n", "lb_get_moments", "lb_reduce",
                 "lb_batch_create", "lb_batch_init", "lb_batch_step_n", "lb_batch_get_moments",
                 "lb_batch_status", "lb_destroy", "lb_batch_destroy", "lb_last_error",
                 "lb_batch_step_subset", "lb_batch_set_equilibrium_device", "lbs_create",
                 "lbs_forward", "lbs_train_step", "lbs_conv", "lbs_wgrad", "lb17_create",
                 "lb17_init_lattice", "lb17_step_n", "lb17_get_moments", "lb17_reduce",
                 "lb17_get_populations", "lb17_set_populations", "lb17_destroy"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers exactly the declared calls
    assert sorted(lbvdw.SIGNATURES) == names


def _bytes(lib, **kw):
    p, fx = lbvdw.make_params(**kw)
    n = ctypes.c_size_t()
    st = lib.lb_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return st, n.value, lib.lb_last_error().decode()


def test_workspace_size_scales_with_precision(lib):
    st32, n32, _ = _bytes(lib, Lx=512, Ly=256, fp32=True)
    st64, n64, _ = _bytes(lib, Lx=512, Ly=256, fp32=False)
    assert st32 == 0 and st64 == 0
    nn = 512 * 256
    # two population buffers dominate: 2 x 9 x nn x (4 | 8) bytes
    assert n32 >= 2 * 9 * nn * 4 and n64 >= 2 * 9 * nn * 8
    assert n64 - n32 == pytest.approx(2 * 9 * nn * 4 + 512 * 4, rel=0.01)


@pytest.mark.parametrize("kw,needle", [
    (dict(Lx=0, Ly=16), "Lx"),
    (dict(Lx=16, Ly=3), "Ly"),
    (dict(Lx=16, Ly=16, tau=0.2), "tau"),
    (dict(Lx=16, Ly=16, T=0.0), "T"),
    (dict(Lx=16, Ly=16, U=0.3), "U"),
    (dict(Lx=16, Ly=16, kappa=-1.0), "kappa"),
    (dict(Lx=16, Ly=16, check_every=-1), "check_every"),
    (dict(Lx=4, Ly=16, fext=[0.0, float("nan"), 0.0, 0.0]), "fext"),
    (dict(Lx=16, Ly=16, N=float("inf")), "N, Q"),
])
def test_invalid_parameters_are_rejected(lib, kw, needle):
    st, _, msg = _bytes(lib, **kw)
    assert st == lbvdw.LB_EINVAL
    assert needle in msg


def test_create_rejects_small_or_misaligned_workspace(lib):
    p, _ = lbvdw.make_params(Lx=32, Ly=16)
    h = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the checks come first
    st = lib.lb_create(ctypes.byref(p), fake, 1024, None, ctypes.byref(h))
    assert st == lbvdw.LB_ENOMEM and "needs" in lib.lb_last_error().decode()
    st = lib.lb_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), 1 << 30, None, ctypes.byref(h))
    assert st == lbvdw.LB_EINVAL and "aligned" in lib.lb_last_error().decode()


def test_null_handles_are_rejected(lib):
    assert lib.lb_step_n(None, 1) == lbvdw.LB_EINVAL
    assert lib.lb_get_moments(None, None, None, None) == lbvdw.LB_EINVAL
    assert lib.lb_destroy(None) == lbvdw.LB_OK
    assert lib.lb_batch_step_n(None, 1) == lbvdw.LB_EINVAL


def test_batch_rejects_mixed_precision(lib):
    arr = (lbvdw.lb_params * 2)()
    arr[0], _ = lbvdw.make_params(Lx=32, Ly=16, fp32=True)
    arr[1], _ = lbvdw.make_params(Lx=32, Ly=16, fp32=False)
    h = ctypes.c_void_p()
    st = lib.lb_batch_create(2, arr, ctypes.c_void_p(1 << 20), 1 << 40, None, ctypes.byref(h))
    assert st == lbvdw.LB_EINVAL and "fp32" in lib.lb_last_error().decode()
    n = ctypes.c_size_t()
    assert lib.lb_batch_workspace_bytes(2, arr, ctypes.byref(n)) == 0
    assert lib.lb_batch_workspace_bytes(0, arr, ctypes.byref(n)) == lbvdw.LB_EINVAL


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_1307_6703_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.lower(), f


def test_surrogate_sizes_and_validation(lib):
    n = ctypes.c_int64()
    assert lib.lbs_param_count(ctypes.byref(n)) == 0
    # 3x3 convolutions 6->48, 4 x 48->48, 48->3, with biases
    assert n.value == (9 * 6 * 48 + 48) + 4 * (9 * 48 * 48 + 48) + (9 * 48 * 3 + 3)
    b_inf, b_tr = ctypes.c_size_t(), ctypes.c_size_t()
    assert lib.lbs_workspace_bytes(4, 128, 256, 0, ctypes.byref(b_inf)) == 0
    assert lib.lbs_workspace_bytes(4, 128, 256, 1, ctypes.byref(b_tr)) == 0
    act = 4 * 128 * 256 * 48 * 2
    assert b_inf.value >= 2 * act and b_tr.value >= 14 * act
    assert lib.lbs_workspace_bytes(0, 128, 256, 0, ctypes.byref(b_inf)) == lbvdw.LB_EINVAL
    # unsupported channel pair and bad mode are rejected before any launch
    st = lib.lbs_conv(0, 8, 32, None, None, None, None, None, None, None, None, 0, 1, 4, 4, 0, None)
    assert st == lbvdw.LB_EINVAL and "channel pair" in lib.lb_last_error().decode()
    st = lib.lbs_conv(7, 8, 48, None, None, None, None, None, None, None, None, 0, 1, 4, 4, 0, None)
    assert st == lbvdw.LB_EINVAL and "mode" in lib.lb_last_error().decode()
    # a bias in the backward mode is refused on the host (placeholder pointers,
    # never dereferenced: every check before it passes, none launches)
    fake = ctypes.c_void_p(1 << 20)
    st = lib.lbs_conv(3, 16, 48, fake, fake, fake, None, fake, fake, None, None, 0, 1, 4, 4, 0, None)
    assert st == lbvdw.LB_EINVAL and "no bias" in lib.lb_last_error().decode()
    st = lib.lbs_wgrad(16, 48, 16, 48, None, None, 1, 4, 4, 1.0, None, 1, None, None, None)
    assert st == lbvdw.LB_EINVAL
    assert lib.lbs_create(1, 4, 4, 0, None, 0, None, None) == lbvdw.LB_EINVAL


def _bytes17(lib, **kw):
    kw.setdefault("y_periodic", True)
    p, fx = lbvdw.make_params(**kw)
    n = ctypes.c_size_t()
    st = lib.lb17_workspace_bytes(ctypes.byref(p), ctypes.byref(n))
    return st, n.value, lib.lb_last_error().decode()


def test_d2q17_workspace_and_lattice(lib):
    st32, n32, _ = _bytes17(lib, Lx=512, Ly=256, fp32=True)
    st64, n64, _ = _bytes17(lib, Lx=512, Ly=256, fp32=False)
    assert st32 == 0 and st64 == 0
    nn = 512 * 256
    # two buffers of 17 planes, plus three FP64 moment planes
    assert n32 >= 2 * 17 * nn * 4 + 3 * nn * 8
    assert n64 - n32 == pytest.approx(2 * 17 * nn * 4, rel=0.01)
    # the library's velocity set and weights are the oracle's
    from oracle import d2q17 as o17
    cx, cy, w, s = lbvdw.lattice17()
    ocx, ocy, ow, os_ = o17.lattice()
    assert (cx == ocx).all() and (cy == ocy).all()
    assert np.abs(w - ow).max() < 1e-15 and abs(s - os_) < 1e-15


@pytest.mark.parametrize("kw,needle", [
    (dict(Lx=16, Ly=16, y_periodic=False), "periodic"),
    (dict(Lx=16, Ly=16, U=0.01), "U must be 0"),
    (dict(Lx=16, Ly=16, regularized=True), "BGK"),
    (dict(Lx=16, Ly=3), "Ly"),
    (dict(Lx=16, Ly=16, tau=0.25), "tau"),
    (dict(Lx=8192, Ly=4096, fp32=True), "2 GiB"),
    (dict(Lx=4, Ly=16, fext=[0.0, float("nan"), 0.0, 0.0]), "fext"),
])
def test_d2q17_invalid_parameters_are_rejected(lib, kw, needle):
    st, _, msg = _bytes17(lib, **kw)
    assert st == lbvdw.LB_EINVAL
    assert needle in msg


def test_d2q17_precision_field(lib):
    for v in (0, 1, 2):
        st, n, _ = _bytes17(lib, Lx=64, Ly=32, fp32=v)
        assert st == 0 and n > 0
    p, _ = lbvdw.make_params(Lx=64, Ly=32, y_periodic=True)
    p.fp32 = 3
    n = ctypes.c_size_t()
    assert lib.lb17_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == lbvdw.LB_EINVAL
    assert "fp32" in lib.lb_last_error().decode()


def test_d2q17_create_checks_the_workspace_first(lib):
    p, _ = lbvdw.make_params(Lx=32, Ly=16, y_periodic=True)
    h = ctypes.c_void_p()
    st = lib.lb17_create(ctypes.byref(p), ctypes.c_void_p(1 << 20), 1024, None, ctypes.byref(h))
    assert st == lbvdw.LB_ENOMEM and "too small" in lib.lb_last_error().decode()
    st = lib.lb17_create(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), 1 << 30, None,
                         ctypes.byref(h))
    assert st == lbvdw.LB_EINVAL and "aligned" in lib.lb_last_error().decode()
    assert lib.lb17_step_n(None, 1) == lbvdw.LB_EINVAL
    assert lib.lb17_destroy(None) == lbvdw.LB_OK
