"""Pins of the oracle's pointwise pieces against what the paper fixes.

Each test checks an oracle function against a property stated by the paper
or by the mathematics (moment identities, consistency conditions, the
critical point), never against a retyped copy of the same code.
"""
import math

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import lb_oracle as lo

SQ3 = math.sqrt(3.0)
DT = 1.0 / SQ3  # the paper's time step (Sec. III)
E = SQ3 * np.stack([lo.CX, lo.CY], axis=1).astype(float)  # paper-unit speeds


def _rng(seed=7):
    return np.random.Generator(np.random.PCG64(seed))


def test_velocity_set_is_gauss_hermite_d2q9():
    # Sec. II: |e| = sqrt(3) on axes, sqrt(6) on diagonals; weights 4/9, 1/9, 1/36.
    speeds = np.linalg.norm(E, axis=1)
    assert np.allclose(speeds, [0] + [SQ3] * 4 + [math.sqrt(6)] * 4)
    assert math.isclose(lo.W.sum(), 1.0, rel_tol=0, abs_tol=1e-15)
    # Gauss-Hermite quadrature: second and fourth lattice moments of the weights
    # equal those of the unit Maxwellian in paper units.
    m2 = np.einsum("i,ia,ib->ab", lo.W, E, E)
    assert np.allclose(m2, np.eye(2), atol=1e-15)
    m4 = np.einsum("i,ia,ib,ic,id->abcd", lo.W, E, E, E, E)
    d = np.eye(2)
    iso = np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) + np.einsum("ad,bc->abcd", d, d)
    assert np.allclose(m4, iso, atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_equilibrium_moments(seed):
    # Sec. II: sum f_eq = n, sum f_eq e = n u, sum f_eq e e = n T I + n u u
    # (paper units). The oracle works in lattice units, u_l = u_p / sqrt(3).
    g = _rng(seed)
    n, T = g.uniform(0.3, 2.0), g.uniform(0.8, 1.0)
    up = g.uniform(-0.2, 0.2, 2)
    f = lo.feq(n, up[0] / SQ3, up[1] / SQ3, T)
    assert abs(f.sum() - n) <= 1e-15 * 4
    assert np.allclose(f @ E, n * up, atol=1e-15, rtol=0)
    m2 = np.einsum("i,ia,ib->ab", f, E, E)
    assert np.allclose(m2, n * T * np.eye(2) + n * np.outer(up, up), atol=4e-15, rtol=0)


@pytest.mark.parametrize("seed", range(5))
def test_forcing_moments_match_coefficients(seed):
    # Eq.(forceterm) with Eq.(coeff): the zeroth, first and second moments of
    # the forcing are A = 0, B = (1 - dt/2tau) F and C (paper units). The oracle
    # takes lattice-unit inputs and returns dt * forcing.
    g = _rng(100 + seed)
    T, tau = g.uniform(0.8, 1.0), g.uniform(0.5, 3.0)
    u = g.uniform(-0.2, 0.2, 2)       # u* (paper units)
    F = g.uniform(-0.05, 0.05, 2)     # force density (paper units)
    gn = g.uniform(-0.2, 0.2, 2)      # grad n
    D = g.uniform(-0.1, 0.1)          # d_gamma (n u*_gamma) (paper units)
    out = lo.forcing(u[0] / SQ3, u[1] / SQ3, F[0] / 3, F[1] / 3, gn[0], gn[1], D / SQ3,
                     T, SQ3 * tau)
    s = 1.0 - DT / (2.0 * tau)
    C = s * (np.outer(u, F) + np.outer(F, u) + (1 - T) * (np.outer(u, gn) + np.outer(gn, u)
                                                          + D * np.eye(2)))
    assert abs(out.sum()) <= 1e-16 * 10
    assert np.allclose(out @ E, DT * s * F, atol=1e-16, rtol=1e-13)
    assert np.allclose(np.einsum("i,ia,ib->ab", out, E, E), DT * C, atol=1e-16, rtol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_collision_changes_momentum_by_force(seed):
    # Eq.(evoleq) with Eq.(newvel): if n u* = sum f c + F/2, the post-collision
    # momentum is sum f c + F (lattice units), for any tau.
    g = _rng(200 + seed)
    T, tau_l = g.uniform(0.85, 1.0), g.uniform(0.6, 4.0)
    n = g.uniform(0.5, 1.5)
    f = lo.feq(n, 0.01, -0.02, T) + g.uniform(-1e-3, 1e-3, 9)
    n = f.sum()
    Fl = g.uniform(-1e-2, 1e-2, 2)
    c = np.stack([lo.CX, lo.CY], axis=1).astype(float)
    j = f @ c + 0.5 * Fl
    u = j / n
    fe = lo.feq(n, u[0], u[1], T)
    fo = lo.forcing(u[0], u[1], Fl[0], Fl[1], 0.1, -0.2, 0.05, T, tau_l)
    S = f - (f - fe) / tau_l + fo
    assert abs(S.sum() - f.sum()) < 1e-15
    assert np.allclose(S @ c - f @ c, Fl, atol=1e-16, rtol=1e-13)


def test_pressure_term_is_ideal_minus_vdw():
    # Eq.(force2): the scalar under the gradient is p^i - p^w with p^i = n T,
    # and Eq.(eqstate) has its critical point at n = T = 1 with p = 3/8.
    pw = lambda n, T: n * T - lo.pressure_term(n, T)
    assert math.isclose(pw(1.0, 1.0), 3.0 / 8.0, rel_tol=0, abs_tol=1e-15)
    h = 1e-4
    d1 = (pw(1 + h, 1.0) - pw(1 - h, 1.0)) / (2 * h)
    d2 = (pw(1 + h, 1.0) - 2 * pw(1.0, 1.0) + pw(1 - h, 1.0)) / h**2
    assert abs(d1) < 1e-8 and abs(d2) < 1e-6
    # p^w = n psi'(n) - psi(n) with the free energy of Sec. II, on a grid.
    for n in np.linspace(0.2, 2.5, 12):
        for T in (0.85, 0.95):
            assert math.isclose(pw(n, T), n * cf.mu(n, T) - cf.psi(n, T), rel_tol=1e-13, abs_tol=1e-14)


def _walls(Lx, Ly, N, Q):
    return lo.Params(Lx, Ly, N=N, Q=Q, y_periodic=False)


@pytest.mark.parametrize("N,Q", [(0.5, 1.0), (0.3, 2.0), (0.4, 2.1), (1.0, 0.0), (0.0, 3.9)])
def test_stencils_exact_on_polynomials(N, Q):
    # Eq.(xstencil), Eq.(laplstencil): 2N + 4M = 1 makes the gradient exact on
    # linear fields and Q + 2R = 1 makes the Laplacian exact on quadratics, for
    # every (N, Q). The y derivative points along +y.
    Lx, Ly = 12, 10
    p = _walls(Lx, Ly, N, Q)
    y, x = np.mgrid[0:Ly, 0:Lx].astype(float)
    inner = (slice(1, Ly - 1), slice(1, Lx - 1))
    gx, gy, lap = lo.stencils(p, 0.3 + 0.7 * x - 1.3 * y)
    assert np.allclose(gx[inner], 0.7, atol=1e-13) and np.allclose(gy[inner], -1.3, atol=1e-13)
    for field, want in ((x * x, 2.0), (y * y, 2.0), (x * y, 0.0), (x * x - y * y, 0.0)):
        _, _, lap = lo.stencils(p, field)
        assert np.allclose(lap[inner], want, atol=1e-11)
    gx, gy, _ = lo.stencils(p, x * y)
    assert np.allclose(gx[inner], y[inner], atol=1e-12)
    assert np.allclose(gy[inner], x[inner], atol=1e-12)


@pytest.mark.parametrize("N,Q", [(0.3, 2.0), (0.4, 2.1), (1.0, 0.0)])
def test_stencils_collapse_on_x_only_fields(N, Q):
    # On a field that varies along x only, the M and R entries fold into the
    # central row, so every (N, Q) gives central differences.
    Lx, Ly = 16, 6
    g = _rng(3)
    row = g.uniform(0.5, 1.5, Lx)
    phi = np.tile(row, (Ly, 1))
    p = lo.Params(Lx, Ly, N=N, Q=Q, y_periodic=True)
    gx, gy, lap = lo.stencils(p, phi)
    assert np.allclose(gx, np.tile(0.5 * (np.roll(row, -1) - np.roll(row, 1)), (Ly, 1)), atol=1e-15)
    assert np.allclose(lap, np.tile(np.roll(row, -1) + np.roll(row, 1) - 2 * row, (Ly, 1)), atol=1e-14)
    assert np.allclose(gy, 0.0, atol=1e-15)


def test_wall_ghosts_give_zero_normal_derivative():
    # Neutral wetting (Sec. II): the normal derivative of n vanishes at the
    # walls, for even fields; odd fields (y-components) keep a normal slope.
    Lx, Ly = 9, 8
    g = _rng(5)
    phi = g.uniform(0.5, 1.5, (Ly, Lx))
    p = _walls(Lx, Ly, 0.3, 2.0)
    _, gy, _ = lo.stencils(p, phi, parity=1.0)
    assert np.allclose(gy[0], 0.0, atol=1e-15) and np.allclose(gy[-1], 0.0, atol=1e-15)
    _, gy_odd, _ = lo.stencils(p, phi, parity=-1.0)
    N, M = 0.3, (1 - 0.6) / 4
    want = 2 * N * phi[1] + 2 * M * (np.roll(phi[1], -1) + np.roll(phi[1], 1))
    assert np.allclose(gy_odd[0], want, atol=1e-14)
