"""ctypes binding of liblbvdw.so (include/lbvdw.h), names as in the C ABI.

Argument marshalling only: every step of the method runs in the HIP kernels of
the library. PyTorch provides device memory (the workspace tensor) and the
stream. If the library is missing the import of this module still works, but
creating a lattice raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbvdw.so")

LB_OK, LB_EINVAL, LB_ENOMEM, LB_EDEVICE, LB_EUNSTABLE, LB_ESTATE = 0, -1, -2, -3, -4, -5
_STATUS = {LB_EINVAL: "LB_EINVAL", LB_ENOMEM: "LB_ENOMEM", LB_EDEVICE: "LB_EDEVICE",
           LB_EUNSTABLE: "LB_EUNSTABLE", LB_ESTATE: "LB_ESTATE"}


class LBError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class lb_params(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("y_periodic", ctypes.c_int32), ("fp32", ctypes.c_int32),
                ("T", ctypes.c_double), ("tau", ctypes.c_double), ("kappa", ctypes.c_double),
                ("N", ctypes.c_double), ("Q", ctypes.c_double), ("U", ctypes.c_double),
                ("fext_x", ctypes.POINTER(ctypes.c_double)),
                ("check_every", ctypes.c_int32), ("drift_correct", ctypes.c_int32),
                ("collision", ctypes.c_int32)]


_DP = ctypes.POINTER(ctypes.c_double)
_VP = ctypes.c_void_p
_I32P = ctypes.POINTER(ctypes.c_int32)
_PP = ctypes.POINTER(lb_params)

# name -> (restype, argtypes); the complete list of exported entry points.
SIGNATURES = {
    "lb_last_error": (ctypes.c_char_p, []),
    "lb_workspace_bytes": (ctypes.c_int, [_PP, ctypes.POINTER(ctypes.c_size_t)]),
    "lb_create": (ctypes.c_int, [_PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lb_init_lattice": (ctypes.c_int, [_VP, _DP, _DP, _DP]),
    "lb_init_lattice_device": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lb_step_n": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "lb_get_moments": (ctypes.c_int, [_VP, _DP, _DP, _DP]),
    "lb_get_moments_device": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lb_reduce": (ctypes.c_int, [_VP, _DP]),
    "lb_get_populations": (ctypes.c_int, [_VP, _DP]),
    "lb_set_populations": (ctypes.c_int, [_VP, _DP, ctypes.c_int64]),
    "lb_get_step": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "lb_set_checks": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb_destroy": (ctypes.c_int, [_VP]),
    "lb_batch_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, _PP, ctypes.POINTER(ctypes.c_size_t)]),
    "lb_batch_create": (ctypes.c_int, [ctypes.c_int32, _PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lb_batch_init": (ctypes.c_int, [_VP, ctypes.c_int32, _DP, _DP, _DP]),
    "lb_batch_step_n": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "lb_batch_get_moments": (ctypes.c_int, [_VP, ctypes.c_int32, _DP, _DP, _DP]),
    "lb_batch_reduce": (ctypes.c_int, [_VP, ctypes.c_int32, _DP]),
    "lb_batch_status": (ctypes.c_int, [_VP, _I32P]),
    "lb_batch_drop_unstable": (ctypes.c_int, [_VP, _I32P]),
    "lb_batch_destroy": (ctypes.c_int, [_VP]),
    "lb_set_launch": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb_get_launch": (ctypes.c_int, [_VP, _I32P, _I32P, _I32P]),
    "lb_set_launch_fused": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb_get_steps_per_launch": (ctypes.c_int, [_VP, _I32P]),
    "lb_batch_set_launch_fused": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb_batch_get_steps_per_launch": (ctypes.c_int, [_VP, _I32P]),
    "lb_batch_set_launch": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb_autotune": (ctypes.c_int, [_VP, ctypes.c_int32, _I32P, _I32P, _DP]),
    "lb_batch_autotune": (ctypes.c_int, [_VP, ctypes.c_int32, _I32P, _I32P, _DP]),
    "lb_batch_get_moments_device": (ctypes.c_int, [_VP, _VP]),
    "lb_batch_set_equilibrium_device": (ctypes.c_int, [_VP, _VP, _I32P]),
    "lb_batch_shift_equilibrium_device": (ctypes.c_int, [_VP, _VP, _VP, _I32P]),
    "lb_batch_step_subset": (ctypes.c_int, [_VP, ctypes.c_int64, _I32P]),
    # include/lbd2q17.h
    "lb17_lattice": (ctypes.c_int, [_I32P, _I32P, _DP, _DP]),
    "lb17_workspace_bytes": (ctypes.c_int, [_PP, ctypes.POINTER(ctypes.c_size_t)]),
    "lb17_create": (ctypes.c_int, [_PP, _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lb17_init_lattice": (ctypes.c_int, [_VP, _DP, _DP, _DP]),
    "lb17_init_lattice_device": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lb17_get_moments_device": (ctypes.c_int, [_VP, _VP, _VP, _VP]),
    "lb17_step_n": (ctypes.c_int, [_VP, ctypes.c_int64]),
    "lb17_get_moments": (ctypes.c_int, [_VP, _DP, _DP, _DP]),
    "lb17_reduce": (ctypes.c_int, [_VP, _DP]),
    "lb17_get_populations": (ctypes.c_int, [_VP, _DP]),
    "lb17_set_populations": (ctypes.c_int, [_VP, _DP, ctypes.c_int64]),
    "lb17_set_launch": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32]),
    "lb17_get_launch": (ctypes.c_int, [_VP, _I32P, _I32P, _I32P]),
    "lb17_get_step": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64)]),
    "lb17_autotune": (ctypes.c_int, [_VP, ctypes.c_int32, _I32P, _I32P, _DP]),
    "lb17_destroy": (ctypes.c_int, [_VP]),
    # include/lbsurrogate.h
    "lbs_param_count": (ctypes.c_int, [ctypes.POINTER(ctypes.c_int64)]),
    "lbs_workspace_bytes": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]),
    "lbs_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  _VP, ctypes.c_size_t, _VP, ctypes.POINTER(_VP)]),
    "lbs_set_params": (ctypes.c_int, [_VP, _VP]),
    "lbs_get_params": (ctypes.c_int, [_VP, _VP]),
    "lbs_get_grads": (ctypes.c_int, [_VP, _VP]),
    "lbs_forward": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP]),
    "lbs_train_step": (ctypes.c_int, [_VP, ctypes.c_int32, _VP, _VP, ctypes.c_float, _VP]),
    "lbs_destroy": (ctypes.c_int, [_VP]),
    "lbs_pack": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, _VP, _VP]),
    "lbs_conv": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP, _VP, _VP, _VP,
                                _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_int32, ctypes.c_int32, _VP]),
    "lbs_wgrad": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                 _VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_float,
                                 _VP, ctypes.c_int32, _VP, _VP, _VP]),
    "lbs_wgrad_scratch_floats": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                                ctypes.c_int32, ctypes.c_int32,
                                                ctypes.POINTER(ctypes.c_int64)]),
    "lbs_wgrad_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, _VP, _VP, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_float, ctypes.c_int32, _VP, _VP,
                                         _VP]),
    "lbs_bias_grad": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_float, _VP, _VP, _VP]),
    "lbs_mse": (ctypes.c_int, [_VP, _VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP, _VP,
                               _VP, _VP]),
    "lbs_adam": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, ctypes.c_int32, _VP]),
    "lbs_fields_to_input": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _VP,
                                           _VP, ctypes.c_int32, _VP, _VP, _VP]),
    "lbs_make_target": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, _VP, _VP, _VP]),
    "lbs_apply_output": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, _VP, _VP, _VP]),
    "lbs_compare": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, _VP, _VP]),
    "lbs_project_mass": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int64, _VP, _VP]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbvdw.so and bind every entry point. Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    # PyTorch ships its own HIP runtime with the same soname; loading torch
    # first makes this library bind to it, so both share one runtime (one set
    # of devices, streams and allocations).
    import torch  # noqa: F401
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1307_6703_amd/build.py "
                           "(hipcc, gfx950); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(st: int):
    if st != LB_OK:
        raise LBError(st, _lib.lb_last_error().decode())


def _dptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(_DP)


def _host(a, shape) -> Optional[np.ndarray]:
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if a.size != int(np.prod(shape)):
        raise ValueError(f"expected {shape} values, got {a.shape}")
    return a.reshape(shape)


def _require(t, dtype, numel: int):
    """A contiguous device tensor of the given dtype and size (the C ABI
    takes its raw pointer)."""
    if t.dtype != dtype or not t.is_contiguous() or t.numel() != numel or not t.is_cuda:
        raise ValueError(f"expected a contiguous {dtype} device tensor of {numel} elements, "
                         f"got {t.dtype} {tuple(t.shape)} on {t.device}")


# lb_params.fp32: FP64 populations; FP32 deviations with FP32 arithmetic; FP32
# deviations with FP64 arithmetic and stochastic rounding of the stored values
FP64, FP32, FP32_SR = 0, 1, 2


def precision(fp32) -> int:
    """lb_params.fp32 from False / True (FP64 / FP32), 0, 1, 2 or "sr"."""
    if isinstance(fp32, str):
        if fp32 != "sr":
            raise ValueError(f"unknown precision {fp32!r}")
        return FP32_SR
    v = int(fp32)
    if v not in (FP64, FP32, FP32_SR):
        raise ValueError(f"fp32 must be 0, 1, 2, False, True or 'sr' (got {fp32!r})")
    return v


def make_params(Lx, Ly, T=0.95, tau=1.0, kappa=0.3, N=0.3, Q=2.0, U=0.0, fext=None,
                y_periodic=False, fp32=False, check_every=0, drift_correct=False,
                regularized=False):
    """Fill an lb_params; returns (params, fext array kept alive by the caller)."""
    fx = _host(fext, (Lx,)) if fext is not None else None
    p = lb_params(int(Lx), int(Ly), int(bool(y_periodic)), precision(fp32), float(T), float(tau),
                  float(kappa), float(N), float(Q), float(U), _dptr(fx), int(check_every),
                  int(bool(drift_correct)), int(bool(regularized)))
    return p, fx


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Lattice:
    """One lattice on the current GPU: workspace tensor + lb_handle."""

    def __init__(self, Lx, Ly, *, T=0.95, tau=1.0, kappa=0.3, N=0.3, Q=2.0, U=0.0, fext=None,
                 y_periodic=False, fp32=False, check_every=0, drift_correct=False,
                 regularized=False, device="cuda", stream=None):
        import torch
        lib = load_library()
        self.Lx, self.Ly = int(Lx), int(Ly)
        self.precision = precision(fp32)
        self.fp32 = self.precision != FP64  # FP32 storage
        self._p, self._fext = make_params(Lx, Ly, T, tau, kappa, N, Q, U, fext, y_periodic, fp32,
                                          check_every, drift_correct, regularized)
        nbytes = ctypes.c_size_t()
        _check(lib.lb_workspace_bytes(ctypes.byref(self._p), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib.lb_create(ctypes.byref(self._p), ctypes.c_void_p(base + off), nbytes.value,
                             _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    @property
    def shape(self):
        return (self.Ly, self.Lx)

    def init(self, n0, ux0=None, uy0=None):
        import torch
        if isinstance(n0, torch.Tensor) and n0.is_cuda:
            t = [None if a is None else a.to(torch.float64).contiguous() for a in (n0, ux0, uy0)]
            self._keep = t
            ptr = lambda a: None if a is None else ctypes.c_void_p(a.data_ptr())
            _check(_lib.lb_init_lattice_device(self._h, ptr(t[0]), ptr(t[1]), ptr(t[2])))
            return self
        a = [_host(v, self.shape) for v in (n0, ux0, uy0)]
        _check(_lib.lb_init_lattice(self._h, _dptr(a[0]), _dptr(a[1]), _dptr(a[2])))
        return self

    def step(self, nsteps: int = 1):
        _check(_lib.lb_step_n(self._h, int(nsteps)))
        return self

    def moments(self):
        n, ux, uy = (np.empty(self.shape) for _ in range(3))
        _check(_lib.lb_get_moments(self._h, _dptr(n), _dptr(ux), _dptr(uy)))
        return n, ux, uy

    def moments_device(self):
        import torch
        out = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.workspace.device)
        ptr = lambda k: ctypes.c_void_p(out[k].data_ptr())
        _check(_lib.lb_get_moments_device(self._h, ptr(0), ptr(1), ptr(2)))
        return out

    def reduce(self):
        out = np.empty(6)
        _check(_lib.lb_reduce(self._h, _dptr(out)))
        return dict(mass=out[0], jx=out[1], jy=out[2], nmin=out[3], nmax=out[4], nonfinite=out[5])

    def populations(self):
        f = np.empty((9,) + self.shape)
        _check(_lib.lb_get_populations(self._h, _dptr(f)))
        return f

    def set_populations(self, f, step: int = 0):
        f = _host(f, (9,) + self.shape)
        _check(_lib.lb_set_populations(self._h, _dptr(f), int(step)))
        return self

    @property
    def step_count(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.lb_get_step(self._h, ctypes.byref(v)))
        return v.value

    def set_launch(self, threads: int = 0, rows: int = 0, steps_per_launch: int = 1):
        """Launch shape; steps_per_launch = 2 selects the two-step kernel
        (FP32 only; threads 64, 128, 192 or 256)."""
        if steps_per_launch == 2:
            _check(_lib.lb_set_launch_fused(self._h, int(threads), int(rows)))
        elif steps_per_launch == 1:
            _check(_lib.lb_set_launch(self._h, int(threads), int(rows)))
        else:
            raise ValueError("steps_per_launch must be 1 or 2")

    def steps_per_launch(self) -> int:
        v = ctypes.c_int32()
        _check(_lib.lb_get_steps_per_launch(self._h, ctypes.byref(v)))
        return v.value

    def set_checks(self, check_every: int, drift_correct: bool = False):
        _check(_lib.lb_set_checks(self._h, int(check_every), int(bool(drift_correct))))

    def get_launch(self):
        t, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lb_get_launch(self._h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(b)))
        return t.value, r.value, b.value

    def autotune(self, nsteps: int = 5):
        t, r, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(_lib.lb_autotune(self._h, int(nsteps), ctypes.byref(t), ctypes.byref(r), ctypes.byref(ms)))
        return t.value, r.value, ms.value

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lattice17():
    """The D2Q17 velocity set: (cx, cy, w, s) as lb17_lattice gives them."""
    load_library()
    cx, cy = (ctypes.c_int32 * 17)(), (ctypes.c_int32 * 17)()
    w = np.empty(17)
    s = ctypes.c_double()
    _check(_lib.lb17_lattice(cx, cy, _dptr(w), ctypes.byref(s)))
    return np.array(cx[:]), np.array(cy[:]), w, s.value


class Lattice17:
    """One periodic D2Q17 lattice on the current GPU (include/lbd2q17.h):
    workspace tensor + lb17_handle. Parameters as for Lattice; y_periodic is
    implied, U must be 0; fp32 as for Lattice (False, True or "sr")."""

    def __init__(self, Lx, Ly, *, T=0.95, tau=1.0, kappa=0.3, N=0.3, Q=2.0, fext=None,
                 fp32=False, check_every=0, drift_correct=False, device="cuda", stream=None):
        import torch
        lib = load_library()
        self.Lx, self.Ly = int(Lx), int(Ly)
        self.precision = precision(fp32)
        self.fp32 = self.precision != FP64  # FP32 storage
        self._p, self._fext = make_params(Lx, Ly, T, tau, kappa, N, Q, 0.0, fext, True,
                                          self.precision, check_every, drift_correct, False)
        nbytes = ctypes.c_size_t()
        _check(lib.lb17_workspace_bytes(ctypes.byref(self._p), ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib.lb17_create(ctypes.byref(self._p), ctypes.c_void_p(base + off), nbytes.value,
                               _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    @property
    def shape(self):
        return (self.Ly, self.Lx)

    def init(self, n0, ux0=None, uy0=None):
        import torch
        if isinstance(n0, torch.Tensor) and n0.is_cuda:
            t = [None if a is None else a.to(torch.float64).contiguous() for a in (n0, ux0, uy0)]
            self._keep = t
            ptr = lambda a: None if a is None else ctypes.c_void_p(a.data_ptr())
            _check(_lib.lb17_init_lattice_device(self._h, ptr(t[0]), ptr(t[1]), ptr(t[2])))
            return self
        a = [_host(v, self.shape) for v in (n0, ux0, uy0)]
        _check(_lib.lb17_init_lattice(self._h, _dptr(a[0]), _dptr(a[1]), _dptr(a[2])))
        return self

    def step(self, nsteps: int = 1):
        _check(_lib.lb17_step_n(self._h, int(nsteps)))
        return self

    def moments(self):
        n, ux, uy = (np.empty(self.shape) for _ in range(3))
        _check(_lib.lb17_get_moments(self._h, _dptr(n), _dptr(ux), _dptr(uy)))
        return n, ux, uy

    def moments_device(self):
        import torch
        out = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.workspace.device)
        ptr = lambda k: ctypes.c_void_p(out[k].data_ptr())
        _check(_lib.lb17_get_moments_device(self._h, ptr(0), ptr(1), ptr(2)))
        return out

    def reduce(self):
        out = np.empty(6)
        _check(_lib.lb17_reduce(self._h, _dptr(out)))
        return dict(mass=out[0], jx=out[1], jy=out[2], nmin=out[3], nmax=out[4], nonfinite=out[5])

    def populations(self):
        f = np.empty((17,) + self.shape)
        _check(_lib.lb17_get_populations(self._h, _dptr(f)))
        return f

    def set_populations(self, f, step: int = 0):
        f = _host(f, (17,) + self.shape)
        _check(_lib.lb17_set_populations(self._h, _dptr(f), int(step)))
        return self

    @property
    def step_count(self) -> int:
        v = ctypes.c_int64()
        _check(_lib.lb17_get_step(self._h, ctypes.byref(v)))
        return v.value

    def set_launch(self, threads: int = 0, rows: int = 0):
        _check(_lib.lb17_set_launch(self._h, int(threads), int(rows)))

    def get_launch(self):
        t, r, b = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib.lb17_get_launch(self._h, ctypes.byref(t), ctypes.byref(r), ctypes.byref(b)))
        return t.value, r.value, b.value

    def autotune(self, nsteps: int = 10):
        t, r, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(_lib.lb17_autotune(self._h, int(nsteps), ctypes.byref(t), ctypes.byref(r),
                                  ctypes.byref(ms)))
        return t.value, r.value, ms.value

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lb17_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Many independent lattices advanced together (lb_batch_*).

    instances: list of dicts with the keyword arguments of Lattice (Lx, Ly,
    T, tau, kappa, N, Q, U, fext, y_periodic); fp32, check_every,
    drift_correct and regularized are shared by all instances."""

    def __init__(self, instances, *, fp32=True, check_every=0, drift_correct=False,
                 regularized=False, device="cuda", stream=None):
        import torch
        lib = load_library()
        self.count = len(instances)
        arr = (lb_params * self.count)()
        self._fext = []
        self.shapes = []
        for i, kw in enumerate(instances):
            kw = dict(kw)
            Lx, Ly = kw.pop("Lx"), kw.pop("Ly")
            p, fx = make_params(Lx, Ly, fp32=fp32, check_every=check_every,
                                drift_correct=drift_correct, regularized=regularized, **kw)
            arr[i] = p
            self._fext.append(fx)
            self.shapes.append((int(Ly), int(Lx)))
        self._arr = arr
        nbytes = ctypes.c_size_t()
        _check(lib.lb_batch_workspace_bytes(self.count, arr, ctypes.byref(nbytes)))
        self.workspace = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        off = (-base) % 256
        h = ctypes.c_void_p()
        _check(lib.lb_batch_create(self.count, arr, ctypes.c_void_p(base + off), nbytes.value,
                                   _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def init(self, idx, n0, ux0=None, uy0=None):
        shp = self.shapes[idx]
        a = [_host(v, shp) for v in (n0, ux0, uy0)]
        _check(_lib.lb_batch_init(self._h, int(idx), _dptr(a[0]), _dptr(a[1]), _dptr(a[2])))

    def step(self, nsteps: int = 1):
        _check(_lib.lb_batch_step_n(self._h, int(nsteps)))
        return self

    def moments(self, idx):
        shp = self.shapes[idx]
        n, ux, uy = (np.empty(shp) for _ in range(3))
        _check(_lib.lb_batch_get_moments(self._h, int(idx), _dptr(n), _dptr(ux), _dptr(uy)))
        return n, ux, uy

    def reduce(self, idx):
        out = np.empty(6)
        _check(_lib.lb_batch_reduce(self._h, int(idx), _dptr(out)))
        return dict(mass=out[0], jx=out[1], jy=out[2], nmin=out[3], nmax=out[4], nonfinite=out[5])

    def status(self):
        out = (ctypes.c_int32 * self.count)()
        _check(_lib.lb_batch_status(self._h, out))
        return list(out)

    def set_launch(self, threads: int = 0, rows: int = 0, steps_per_launch: int = 1):
        """Launch shape shared by all instances; steps_per_launch = 2 selects
        the two-step kernel (FP32 only; threads 64, 128, 192 or 256)."""
        if steps_per_launch == 2:
            _check(_lib.lb_batch_set_launch_fused(self._h, int(threads), int(rows)))
        elif steps_per_launch == 1:
            _check(_lib.lb_batch_set_launch(self._h, int(threads), int(rows)))
        else:
            raise ValueError("steps_per_launch must be 1 or 2")

    def steps_per_launch(self) -> int:
        v = ctypes.c_int32()
        _check(_lib.lb_batch_get_steps_per_launch(self._h, ctypes.byref(v)))
        return v.value

    def drop_unstable(self) -> int:
        """Take instances that failed a check out of the steps; returns how
        many have been dropped so far."""
        n = ctypes.c_int32()
        _check(_lib.lb_batch_drop_unstable(self._h, ctypes.byref(n)))
        return n.value

    def _mask(self, mask):
        m = np.ascontiguousarray(np.asarray(mask, dtype=np.int32).reshape(-1))
        if m.size != self.count:
            raise ValueError(f"mask needs {self.count} entries, got {m.size}")
        return m, m.ctypes.data_as(_I32P)

    def moments_device(self, out=None):
        """Moments of every instance (same size) as a device FP64 tensor
        [count, 3, Ly, Lx] (asynchronous on the batch's stream)."""
        import torch
        Ly, Lx = self.shapes[0]
        if out is None:
            out = torch.empty((self.count, 3, Ly, Lx), dtype=torch.float64, device=self.workspace.device)
        _require(out, torch.float64, self.count * 3 * Ly * Lx)
        _check(_lib.lb_batch_get_moments_device(self._h, ctypes.c_void_p(out.data_ptr())))
        return out

    def set_equilibrium(self, fields, mask):
        """Re-enter the instances with mask != 0 as equilibrium populations of
        the device FP64 fields [count, 3, Ly, Lx]."""
        import torch
        Ly, Lx = self.shapes[0]
        _require(fields, torch.float64, self.count * 3 * Ly * Lx)
        m, mp = self._mask(mask)
        _check(_lib.lb_batch_set_equilibrium_device(self._h, ctypes.c_void_p(fields.data_ptr()), mp))

    def shift_equilibrium(self, frm, fields, mask):
        """Re-enter the instances with mask != 0 at the device FP64 fields
        [count, 3, Ly, Lx] keeping their non-equilibrium part: add
        f_eq(fields) - f_eq(frm) to their populations."""
        import torch
        Ly, Lx = self.shapes[0]
        _require(frm, torch.float64, self.count * 3 * Ly * Lx)
        _require(fields, torch.float64, self.count * 3 * Ly * Lx)
        m, mp = self._mask(mask)
        _check(_lib.lb_batch_shift_equilibrium_device(self._h, ctypes.c_void_p(frm.data_ptr()),
                                                      ctypes.c_void_p(fields.data_ptr()), mp))

    def step_subset(self, nsteps: int, mask):
        """Advance only the instances with mask != 0 by an even number of steps."""
        m, mp = self._mask(mask)
        _check(_lib.lb_batch_step_subset(self._h, int(nsteps), mp))
        return self

    def autotune(self, nsteps: int = 5):
        t, r, ms = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_double()
        _check(_lib.lb_batch_autotune(self._h, int(nsteps), ctypes.byref(t), ctypes.byref(r),
                                      ctypes.byref(ms)))
        return t.value, r.value, ms.value

    @property
    def nodes(self) -> int:
        return sum(a * b for a, b in self.shapes)

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.lb_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
