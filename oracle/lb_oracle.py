"""Python front of the FP64 oracle (test infrastructure only).

Loads ``liblb_oracle.so`` (plain C, built by ``oracle/build.py``) and exposes
the step, the initial state and the pointwise pieces (equilibrium of
Eq.(eqfunc), forcing of Eq.(forceterm)/Eq.(coeff), pressure term of
Eq.(force2)/Eq.(eqstate), the stencils of Eq.(xstencil)/Eq.(laplstencil)) so
that tests can pin each of them separately. Everything is in lattice units
(dx = dt = 1); ``tau`` and ``kappa`` are given in the paper's units.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product library never imports it.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

_LIB = None

# D2Q9 velocity set in the order 0 rest, E, N, W, S, NE, NW, SW, SE (Sec. II).
CX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
CY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
W = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


class _Params(ctypes.Structure):
    _fields_ = [("Lx", ctypes.c_int32), ("Ly", ctypes.c_int32),
                ("y_periodic", ctypes.c_int32), ("collision", ctypes.c_int32),
                ("T", ctypes.c_double), ("tau", ctypes.c_double),
                ("kappa", ctypes.c_double), ("N", ctypes.c_double),
                ("Q", ctypes.c_double), ("U", ctypes.c_double)]


def _lib():
    global _LIB
    if _LIB is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(_Params)
        lib.lbo_feq.argtypes = [ctypes.c_double] * 4 + [dp]
        lib.lbo_forcing.argtypes = [ctypes.c_double] * 9 + [dp]
        lib.lbo_regularize.argtypes = [dp, dp]
        lib.lbo_pressure_term.argtypes = [ctypes.c_double, ctypes.c_double]
        lib.lbo_pressure_term.restype = ctypes.c_double
        lib.lbo_apply_stencils.argtypes = [pp, dp, ctypes.c_double, dp, dp, dp]
        lib.lbo_divergence.argtypes = [pp, dp, dp, dp]
        lib.lbo_init.argtypes = [pp, dp, dp, dp, dp]
        lib.lbo_step.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        lib.lbo_step.restype = ctypes.c_int
        lib.lbo_run.argtypes = [pp, dp, dp, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        lib.lbo_run.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Params:
    """Run parameters. Lx, Ly in nodes; U, fext in lattice/paper units as
    documented in the C source; N, Q select the stencil (M, R follow)."""
    Lx: int
    Ly: int
    T: float = 0.95
    tau: float = 1.0
    kappa: float = 0.3
    N: float = 0.3
    Q: float = 2.0
    U: float = 0.0
    y_periodic: bool = False
    regularized: bool = False  # collision of the non-equilibrium part's projection

    def c(self) -> _Params:
        return _Params(self.Lx, self.Ly, int(self.y_periodic), int(bool(self.regularized)),
                       self.T, self.tau, self.kappa, self.N, self.Q, self.U)

    @property
    def tau_l(self) -> float:
        return math.sqrt(3.0) * self.tau


def feq(n, ux, uy, T):
    out = np.zeros(9)
    _lib().lbo_feq(n, ux, uy, T, _ptr(out))
    return out


def regularize(h):
    """Projection of a population vector onto the Hermite polynomials of
    order <= 2 (lbo_regularize)."""
    h = np.ascontiguousarray(h, dtype=np.float64)
    out = np.zeros(9)
    _lib().lbo_regularize(_ptr(h), _ptr(out))
    return out


def forcing(ux, uy, Fx, Fy, dnx, dny, D, T, tau_l):
    out = np.zeros(9)
    _lib().lbo_forcing(ux, uy, Fx, Fy, dnx, dny, D, T, tau_l, _ptr(out))
    return out


def pressure_term(n, T):
    return _lib().lbo_pressure_term(n, T)


def stencils(p: Params, phi: np.ndarray, parity: float = 1.0):
    """Return (d/dx, d/dy, laplacian) of a [Ly, Lx] field with the run's
    boundary handling (periodic or mirrored ghosts of the given parity)."""
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    gx, gy, lap = (np.zeros_like(phi) for _ in range(3))
    c = p.c()
    _lib().lbo_apply_stencils(ctypes.byref(c), _ptr(phi), parity, _ptr(gx), _ptr(gy), _ptr(lap))
    return gx, gy, lap


def divergence(p: Params, jx: np.ndarray, jy: np.ndarray) -> np.ndarray:
    """D = div(j*) of a [Ly, Lx] momentum field as the step computes it."""
    jx = np.ascontiguousarray(jx, dtype=np.float64)
    jy = np.ascontiguousarray(jy, dtype=np.float64)
    D = np.zeros_like(jx)
    c = p.c()
    _lib().lbo_divergence(ctypes.byref(c), _ptr(jx), _ptr(jy), _ptr(D))
    return D


class OracleLB:
    """A lattice held by the oracle: populations S[9, Ly, Lx] (FP64)."""

    def __init__(self, p: Params, n0, ux0=None, uy0=None, fext=None):
        self.p = p
        self._c = p.c()
        n0 = np.ascontiguousarray(n0, dtype=np.float64).reshape(p.Ly, p.Lx)
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64).reshape(p.Ly, p.Lx)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64).reshape(p.Ly, p.Lx)
        self.fext = None if fext is None else np.ascontiguousarray(fext, dtype=np.float64).reshape(p.Lx)
        self.S = np.zeros((9, p.Ly, p.Lx))
        _lib().lbo_init(ctypes.byref(self._c), _ptr(n0), _ptr(ux0), _ptr(uy0), _ptr(self.S))
        self.n = self.ux = self.uy = None
        self.steps = 0

    def run(self, steps: int, threads: int = 0) -> int:
        """Advance `steps` steps; keep the moments of the last one. Returns the
        number of host threads the oracle used."""
        p = self.p
        self.n = np.zeros((p.Ly, p.Lx))
        self.ux = np.zeros((p.Ly, p.Lx))
        self.uy = np.zeros((p.Ly, p.Lx))
        used = _lib().lbo_run(ctypes.byref(self._c), _ptr(self.fext), _ptr(self.S), steps,
                              _ptr(self.n), _ptr(self.ux), _ptr(self.uy), threads)
        if used < 0:
            raise RuntimeError("oracle step failed (bad parameters or out of memory)")
        self.steps += steps
        return used

    def step_into(self, S_out, n=None, ux=None, uy=None) -> None:
        """One step from self.S into S_out without changing self.S."""
        rc = _lib().lbo_step(ctypes.byref(self._c), _ptr(self.fext), _ptr(self.S), _ptr(S_out),
                             _ptr(n), _ptr(ux), _ptr(uy))
        if rc != 0:
            raise RuntimeError("oracle step failed")

    def mass(self) -> float:
        return float(self.S.sum())

    def density(self) -> np.ndarray:
        """Zeroth moment of the stored post-collision populations per node."""
        return self.S.sum(axis=0)
