"""Closed forms of the paper's model, in FP64 (test infrastructure only).

Thermodynamics is in the paper's reduced units (n in units of n_c, T of T_c,
pressure in units of n_c T_c as the paper writes it); flows are in lattice
units. Each function names the passage it follows.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import quad
from scipy.optimize import brentq


# ---- van der Waals fluid (Sec. II, free energy and Eq.(eqstate)) ---------

def psi(n, T):
    """Bulk free-energy density psi = n T ln(3n/(3-n)) - 9 n^2 / 8."""
    return n * T * np.log(3.0 * n / (3.0 - n)) - 9.0 / 8.0 * n * n


def mu(n, T):
    """Chemical potential d psi / d n = T ln(3n/(3-n)) + 3T/(3-n) - 9n/4."""
    return T * np.log(3.0 * n / (3.0 - n)) + 3.0 * T / (3.0 - n) - 9.0 / 4.0 * n


def p_vdw(n, T):
    """Eq.(eqstate): p^w = n psi' - psi = 3 n T / (3 - n) - 9 n^2 / 8."""
    return 3.0 * n * T / (3.0 - n) - 9.0 / 8.0 * n * n


def cs2(n, T):
    """Squared speed of sound d p^w / d n = 9T/(3-n)^2 - 9n/4 (Sec. III)."""
    return 9.0 * T / (3.0 - n) ** 2 - 9.0 / 4.0 * n


def spinodal(T):
    """Densities where d p^w / d n = 0 (T < 1)."""
    lo = brentq(lambda n: cs2(n, T), 1e-6, 1.0)
    hi = brentq(lambda n: cs2(n, T), 1.0, 2.999)
    return lo, hi


def maxwell(T):
    """Coexisting (n_L, n_V, p_coex) at T < 1: equal pressure and equal
    chemical potential (the Maxwell construction of Sec. III). Solved as a
    one-dimensional root in the pressure p: for each p between the spinodal
    pressures, n_V(p) and n_L(p) are the outer branches of p^w(n) = p, and
    mu(n_L(p)) - mu(n_V(p)) changes sign once."""
    if not 0.0 < T < 1.0:
        raise ValueError("coexistence needs 0 < T < 1")
    lo, hi = spinodal(T)
    p_lo = max(p_vdw(hi, T), 1e-14)
    p_hi = p_vdw(lo, T)

    def branches(p):
        nv = brentq(lambda n: p_vdw(n, T) - p, 0.0, lo, xtol=1e-16, rtol=1e-15)
        nl = brentq(lambda n: p_vdw(n, T) - p, hi, 3.0 - 1e-12, xtol=1e-16, rtol=1e-15)
        return nl, nv

    def dmu(p):
        nl, nv = branches(p)
        return mu(nl, T) - mu(nv, T)

    eps = 1e-12 * (p_hi - p_lo)
    pc = brentq(dmu, p_lo + eps, p_hi - eps, xtol=1e-16, rtol=1e-15)
    nl, nv = branches(pc)
    return float(nl), float(nv), float(pc)


def grand_excess(n, T, mu_c, p_c):
    """W(n) = psi(n) - mu_c n + p_c >= 0, zero at both bulk phases."""
    return psi(n, T) - mu_c * n + p_c


def surface_tension(T, kappa):
    """Flat-interface tension sigma = int_{n_V}^{n_L} sqrt(2 kappa W(n)) dn,
    from the square-gradient free energy with kappa (Sec. II)."""
    nl, nv, pc = maxwell(T)
    mc = mu(nl, T)
    val, _ = quad(lambda n: math.sqrt(max(2.0 * kappa * grand_excess(n, T, mc, pc), 0.0)),
                  nv, nl, epsabs=1e-13, epsrel=1e-12, limit=400)
    return val


def interface_profile(T, kappa, x):
    """Exact planar profile n(x) of the square-gradient model (first integral
    kappa n'^2 / 2 = W(n)), centred where n = (n_L + n_V)/2, liquid at +x."""
    nl, nv, pc = maxwell(T)
    mc = mu(nl, T)
    nmid = 0.5 * (nl + nv)

    def pos(n):
        f = lambda m: math.sqrt(kappa / (2.0 * max(grand_excess(m, T, mc, pc), 1e-300)))
        v, _ = quad(f, nmid, n, limit=400)
        return v

    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    out = np.empty_like(x)
    eps = 1e-9
    for k, xv in enumerate(x):
        a, b = nv + eps * (nl - nv), nl - eps * (nl - nv)
        if xv >= pos(b):
            out[k] = b
        elif xv <= pos(a):
            out[k] = a
        else:
            out[k] = brentq(lambda n: pos(n) - xv, a, b, xtol=1e-13)
    return out


def tanh_profile(T, kappa, x):
    """Approximate profile Eq.(interface): n_V + (n_L - n_V)/2 [1 + tanh(x/w)],
    w = sqrt(2 kappa / (1/T - 1))."""
    nl, nv, _ = maxwell(T)
    w = math.sqrt(2.0 * kappa / (1.0 / T - 1.0))
    return nv + 0.5 * (nl - nv) * (1.0 + np.tanh(np.asarray(x) / w))


# ---- flows (lattice units) -------------------------------------------------

def tau_lattice(tau_paper):
    """Relaxation time in steps: the paper's dt is sqrt(3)/3 (Sec. III)."""
    return math.sqrt(3.0) * tau_paper


def kinematic_viscosity(tau_paper):
    """nu = eta / n = tau - dt/2 in paper units (Sec. II, after Eq.(nav)),
    i.e. nu_l = (tau_l - 1/2) / 3 in lattice units."""
    return (tau_lattice(tau_paper) - 0.5) / 3.0


def couette(Ly, U):
    """Steady single-phase Couette flow between wall nodes y = 0 (speed -U)
    and y = Ly - 1 (speed +U): u_x(y) = -U + 2 U y / (Ly - 1)."""
    y = np.arange(Ly, dtype=np.float64)
    return -U + 2.0 * U * y / (Ly - 1)


def two_layer_couette(Ly, U, n_l, n_u):
    """Steady Couette flow of two layers of densities n_l (lower half) and
    n_u (upper half) with equal kinematic viscosity, so the dynamic viscosity
    is proportional to n (Sec. IV, broken-line law). H = Ly - 1 is the gap
    between the wall nodes; the interface sits at H/2. Returns u_x(y)/U."""
    H = Ly - 1.0
    y = np.arange(Ly, dtype=np.float64)
    s = n_l + n_u
    return np.where(y <= H / 2, 4.0 * n_u * y / (H * s) - 1.0,
                    1.0 - 4.0 * n_l * (H - y) / (H * s))


def shear_wave_rate(tau_paper, L):
    """Decay rate per step of u_x = u0 sin(2 pi y / L): nu_l k^2."""
    k = 2.0 * math.pi / L
    return kinematic_viscosity(tau_paper) * k * k


def laplace_dp(sigma, R):
    """Pressure jump across a circular interface in d = 2: sigma / R."""
    return sigma / R
