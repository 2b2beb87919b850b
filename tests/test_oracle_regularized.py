"""Pins of the oracle's regularised collision (Sec. II names the step that
re-projects the post-collision populations onto the Hermite space; the paper
leaves it out at its Knudsen numbers). The projection is checked against what
defines it: it keeps the moments of order 0, 1 and 2, removes the two
third-order and the fourth-order Hermite moments that D2Q9 also carries, is
idempotent and exact on its space. The whole step is checked against BGK
where the two must agree (omega = 1, where nothing of f - f_eq survives) and
against the closed forms the BGK step is pinned to: mass conservation,
the Couette profile and the shear-wave viscosity."""
import math

import numpy as np
import pytest

import lbsynth as ls
from oracle import closed_forms as cf
from oracle.lb_oracle import CX, CY, W, OracleLB, Params, regularize

# the moments the projection keeps: orders 0, 1, 2
KEPT = [np.ones(9), CX, CY, CX * CX, CY * CY, CX * CY]
# the D2Q9 Hermite polynomials of order 3 and 4 (orthogonal to the above
# under the weights W)
DROPPED = [CX * (CY * CY - 1 / 3), CY * (CX * CX - 1 / 3), (CX * CX - 1 / 3) * (CY * CY - 1 / 3)]


def _rng(s):
    return np.random.Generator(np.random.PCG64(s))


def test_dropped_polynomials_are_orthogonal_to_the_kept_ones():
    # the basis the pins below rely on (D2Q9 weights, Sec. II)
    for d in DROPPED:
        for k in KEPT:
            assert abs(np.sum(W * d * k)) < 1e-15


@pytest.mark.parametrize("seed", range(5))
def test_projection_keeps_orders_0_to_2_and_removes_3_and_4(seed):
    h = _rng(seed).normal(size=9)
    p = regularize(h)
    for k in KEPT:
        assert abs(np.sum(p * k) - np.sum(h * k)) < 1e-14
    for d in DROPPED:
        assert abs(np.sum(p * d)) < 1e-14
    # and the difference lies wholly in the dropped part: h - p is a
    # combination of W * DROPPED
    A = np.stack([W * d for d in DROPPED], axis=1)
    coef, *_ = np.linalg.lstsq(A, h - p, rcond=None)
    assert np.abs(A @ coef - (h - p)).max() < 1e-14


def test_projection_is_idempotent_and_exact_on_its_space():
    g = _rng(7)
    h = g.normal(size=9)
    p = regularize(h)
    assert np.abs(regularize(p) - p).max() < 1e-15
    # a vector of the Hermite space (what BGK's f_eq and forcing are made of)
    b0, bx, by, bxx, byy, bxy = g.normal(size=6)
    v = W * (b0 + 3 * (bx * CX + by * CY) +
             4.5 * (bxx * (CX * CX - 1 / 3) + byy * (CY * CY - 1 / 3) + 2 * bxy * CX * CY))
    assert np.abs(regularize(v) - v).max() < 1e-15
    # and the dropped part alone projects to zero
    for d in DROPPED:
        assert np.abs(regularize(W * d)).max() < 1e-16


def _two_phase(p, seed=3, steps=0):
    o = OracleLB(p, ls.noisy_density(p.Lx, p.Ly, seed), fext=ls.potential_force(p.Lx, 0.1, 2))
    if steps:
        o.run(steps, threads=2)
    return o


@pytest.mark.parametrize("periodic", [False, True])
def test_omega_one_equals_bgk(periodic):
    # tau_l = sqrt(3) tau = 1: BGK keeps nothing of f - f_eq, so projecting it
    # first changes nothing (sheared walls, periodic force, two phases forming)
    tau = 1 / math.sqrt(3)
    kw = dict(T=0.95, tau=tau, N=0.3, Q=2.0, U=0.03, y_periodic=periodic)
    a = _two_phase(Params(40, 20, **kw), steps=30)
    b = _two_phase(Params(40, 20, regularized=True, **kw), steps=30)
    assert np.abs(a.S - b.S).max() < 1e-15


@pytest.mark.parametrize("periodic", [False, True])
def test_regularised_step_differs_from_bgk_and_conserves_mass(periodic):
    kw = dict(T=0.95, tau=1.0, N=0.3, Q=2.0, U=0.03, y_periodic=periodic)
    a = _two_phase(Params(48, 24, **kw), steps=200)
    b = _two_phase(Params(48, 24, regularized=True, **kw))
    m0 = b.mass()
    b.run(200, threads=2)
    assert abs(b.mass() - m0) / m0 < 1e-13
    assert np.abs(a.S - b.S).max() > 1e-6  # the projection does something


def test_regularised_couette_profile():
    # Sec. IV flow between the moving walls, as for BGK
    Ly, U = 16, 0.01
    p = Params(3, Ly, T=0.95, N=0.3, Q=2.0, U=U, regularized=True)
    o = OracleLB(p, np.full((Ly, 3), 0.5))
    tS = (Ly - 1) ** 2 / (cf.kinematic_viscosity(1.0) * math.pi**2)
    o.run(int(40 * tS))
    assert np.abs(o.ux - cf.couette(Ly, U)[:, None]).max() < 1e-10
    assert np.abs(o.uy).max() < 1e-12


def _shear_wave_rate(L, tau):
    p = Params(1, L, T=0.95, tau=tau, N=0.3, Q=2.0, y_periodic=True, regularized=True)
    y = np.arange(L)
    s = np.sin(2 * math.pi * y / L)
    o = OracleLB(p, np.full((L, 1), 0.5), ux0=1e-5 * s[:, None])
    o.run(40)
    a1 = o.ux[:, 0] @ s
    o.run(200)
    a2 = o.ux[:, 0] @ s
    return math.log(a1 / a2) / 200


@pytest.mark.parametrize("tau", [1.0, 2.0])
def test_regularised_shear_wave_viscosity(tau):
    # the projection keeps the second moment of f - f_eq, which carries the
    # shear stress, so the viscosity nu_l = (tau_l - 1/2)/3 of Sec. II stays
    r128, r256 = _shear_wave_rate(128, tau), _shear_wave_rate(256, tau)
    e256 = r256 / cf.shear_wave_rate(tau, 256) - 1
    assert abs(e256) < 2e-3
    extrap = (4 * r256 - r128 / 4) / 3 / cf.shear_wave_rate(tau, 256) - 1
    assert abs(extrap) < 5e-5
