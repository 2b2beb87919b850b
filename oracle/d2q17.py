"""Python front of the FP64 D2Q17 oracle (test infrastructure only).

The third-order model with seventeen velocities that the paper names after
Eq.(nav) as the way to remove the u*^3 term of its Navier-Stokes equation,
with the paper's force, stencils and step; ``d2q17_oracle.c`` derives the
lattice, the equilibrium and the forcing term. Periodic lattices only.
Everything is in lattice units; ``tau`` and ``kappa`` are in the paper's units
(``Params`` of ``lb_oracle``).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module; the product library never imports it.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np

from .lb_oracle import Params, _lib, _ptr

_READY = False


def _l():
    global _READY
    lib = _lib()
    if not _READY:
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        pp = ctypes.c_void_p
        lib.lbo17_lattice.argtypes = [ip, ip, dp, dp]
        lib.lbo17_feq.argtypes = [ctypes.c_double] * 4 + [dp]
        lib.lbo17_forcing.argtypes = [ctypes.c_double] * 6 + [dp]
        lib.lbo17_init.argtypes = [pp, dp, dp, dp, dp]
        lib.lbo17_init.restype = ctypes.c_int
        lib.lbo17_step.argtypes = [pp, dp, dp, dp, dp, dp, dp]
        lib.lbo17_step.restype = ctypes.c_int
        lib.lbo17_run.argtypes = [pp, dp, dp, ctypes.c_int64, dp, dp, dp, ctypes.c_int]
        lib.lbo17_run.restype = ctypes.c_int
        _READY = True
    return lib


def lattice():
    """(cx, cy, w, s): integer velocity components, weights, scale s = r^2."""
    cx = (ctypes.c_int * 17)()
    cy = (ctypes.c_int * 17)()
    w = np.zeros(17)
    s = ctypes.c_double()
    _l().lbo17_lattice(cx, cy, _ptr(w), ctypes.byref(s))
    return np.array(cx[:]), np.array(cy[:]), w, s.value


def tau_lattice(tau: float) -> float:
    """Relaxation time in lattice units: tau_l = r tau."""
    return math.sqrt(lattice()[3]) * tau


def feq(n, ux, uy, T):
    out = np.zeros(17)
    _l().lbo17_feq(n, ux, uy, T, _ptr(out))
    return out


def forcing(ux, uy, Fx, Fy, T, tau_l):
    out = np.zeros(17)
    _l().lbo17_forcing(ux, uy, Fx, Fy, T, tau_l, _ptr(out))
    return out


class Oracle17:
    """A periodic D2Q17 lattice held by the oracle: S[17, Ly, Lx] (FP64)."""

    def __init__(self, p: Params, n0, ux0=None, uy0=None, fext=None):
        if not p.y_periodic or p.regularized:
            raise ValueError("the D2Q17 oracle is periodic in y and BGK only")
        self.p = p
        self._c = p.c()
        shp = (p.Ly, p.Lx)
        n0 = np.ascontiguousarray(n0, dtype=np.float64).reshape(shp)
        ux0 = None if ux0 is None else np.ascontiguousarray(ux0, dtype=np.float64).reshape(shp)
        uy0 = None if uy0 is None else np.ascontiguousarray(uy0, dtype=np.float64).reshape(shp)
        self.fext = None if fext is None else \
            np.ascontiguousarray(fext, dtype=np.float64).reshape(p.Lx)
        self.S = np.zeros((17, p.Ly, p.Lx))
        if _l().lbo17_init(ctypes.byref(self._c), _ptr(n0), _ptr(ux0), _ptr(uy0),
                           _ptr(self.S)) != 0:
            raise ValueError("bad parameters")
        self.n = self.ux = self.uy = None
        self.steps = 0

    def run(self, steps: int, threads: int = 0) -> int:
        p = self.p
        self.n = np.zeros((p.Ly, p.Lx))
        self.ux = np.zeros((p.Ly, p.Lx))
        self.uy = np.zeros((p.Ly, p.Lx))
        used = _l().lbo17_run(ctypes.byref(self._c), _ptr(self.fext), _ptr(self.S), steps,
                              _ptr(self.n), _ptr(self.ux), _ptr(self.uy), threads)
        if used < 0:
            raise RuntimeError("oracle step failed")
        self.steps += steps
        return used

    def step_into(self, S_out, n=None, ux=None, uy=None) -> None:
        rc = _l().lbo17_step(ctypes.byref(self._c), _ptr(self.fext), _ptr(self.S), _ptr(S_out),
                             _ptr(n), _ptr(ux), _ptr(uy))
        if rc != 0:
            raise RuntimeError("oracle step failed")

    def mass(self) -> float:
        return float(self.S.sum())

    def momentum(self):
        cx, cy, _, _ = lattice()
        return (float(np.tensordot(cx, self.S, 1).sum()), float(np.tensordot(cy, self.S, 1).sum()))
