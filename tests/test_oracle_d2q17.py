"""Pins of the D2Q17 oracle (CPU only): the third-order model the paper names
after Eq.(nav) to remove the u*^3 term of its Navier-Stokes equation.

Each test checks the oracle against something the mathematics fixes
independently of how the oracle is written: the moments of the unit Gaussian,
the moments of the Maxwellian at temperature T, the shear viscosity a
Chapman-Enskog expansion gives, Galilean invariance (which D2Q9 breaks by the
u*^3 term, as the closed form below predicts), conservation, symmetry, and the
D2Q9 model's own coexistence densities."""
import math

import numpy as np
import pytest

import lbsynth as ls
from oracle import closed_forms as cf
from oracle import d2q17 as o17
from oracle.lb_oracle import CY, OracleLB, Params

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _dfact(k):
    return math.prod(range(k - 1, 0, -2)) if k % 2 == 0 else 0


def test_lattice_is_a_degree_seven_quadrature_of_the_gaussian():
    cx, cy, w, s = o17.lattice()
    assert len(set(zip(cx, cy))) == 17 and (w > 0).all()
    assert max(np.abs(cx).max(), np.abs(cy).max()) == 3
    xi, eta = math.sqrt(s) * cx, math.sqrt(s) * cy
    for a in range(8):
        for b in range(8 - a):
            m = float((w * xi ** a * eta ** b).sum())
            assert abs(m - _dfact(a) * _dfact(b)) < 1e-12, (a, b, m)
    # and not of degree 8: the set is the smallest of this family
    assert abs(float((w * xi ** 8).sum()) - 105) > 1.0


def _sym3(a, M):
    """a_alpha M_beta,gamma summed over the three placements of a."""
    return (np.einsum("a,bc->abc", a, M) + np.einsum("b,ac->abc", a, M) +
            np.einsum("c,ab->abc", a, M))


def _moments(f):
    cx, cy, _, _ = o17.lattice()
    c = np.stack([cx, cy]).astype(float)
    return (f.sum(), c @ f, np.einsum("ai,bi,i->ab", c, c, f),
            np.einsum("ai,bi,ci,i->abc", c, c, c, f))


@pytest.mark.parametrize("seed", range(4))
def test_equilibrium_has_the_maxwellian_moments_to_third_order(seed):
    g = np.random.default_rng(seed)
    n, T = 0.2 + 1.5 * g.random(), 0.8 + 0.5 * g.random()
    u = 0.15 * g.standard_normal(2)
    th = T / o17.lattice()[3]
    M0, M1, M2, M3 = _moments(o17.feq(n, u[0], u[1], T))
    I = np.eye(2)
    assert abs(M0 - n) < 1e-14
    assert np.abs(M1 - n * u).max() < 1e-14
    assert np.abs(M2 - n * (np.outer(u, u) + th * I)).max() < 1e-14
    assert np.abs(M3 - n * (np.einsum("a,b,c->abc", u, u, u) + th * _sym3(u, I))).max() < 1e-14


@pytest.mark.parametrize("seed", range(4))
def test_forcing_term_moments(seed):
    # the rate of change of the Maxwellian's moments under the force alone,
    # times 1 - 1/(2 tau_l): 0, F, u F + F u, F u u + u F u + u u F + theta (F I + ...)
    g = np.random.default_rng(10 + seed)
    T, tau_l = 0.8 + 0.5 * g.random(), 0.6 + g.random()
    u, F = 0.15 * g.standard_normal(2), 1e-3 * g.standard_normal(2)
    th = T / o17.lattice()[3]
    pre = 1 - 0.5 / tau_l
    M0, M1, M2, M3 = _moments(o17.forcing(u[0], u[1], F[0], F[1], T, tau_l))
    uu = np.outer(u, u)
    assert abs(M0) < 1e-18
    assert np.abs(M1 - pre * F).max() < 1e-18
    assert np.abs(M2 - pre * (np.outer(u, F) + np.outer(F, u))).max() < 1e-18
    assert np.abs(M3 - pre * (_sym3(F, uu) + th * _sym3(F, np.eye(2)))).max() < 1e-18


def _shear_rate(model, L, T, tau, U=0.0, n0=0.3, steps=400, amp=1e-5):
    """Decay rate per step of a transverse wave u_y = amp sin(2 pi x / L) on a
    uniform fluid moving at U along x (complex amplitude of the mode, so the
    advection drops out)."""
    Ly = 4
    p = Params(L, Ly, T=T, tau=tau, kappa=0.0, N=0.3, Q=2.0, y_periodic=True)
    x = np.arange(L)
    n = np.full((Ly, L), n0)
    ux = np.full((Ly, L), U)
    uy = np.tile(amp * np.sin(2 * np.pi * x / L), (Ly, 1))
    o = (o17.Oracle17 if model == 17 else OracleLB)(p, n, ux, uy)
    cyv = o17.lattice()[1] if model == 17 else CY

    def mode():
        v = (np.tensordot(cyv, o.S, 1) / o.S.sum(0)).mean(0)
        return abs((v * np.exp(-2j * np.pi * x / L)).sum())

    o.run(20)
    a0 = mode()
    o.run(steps)
    return -math.log(mode() / a0) / steps


@pytest.mark.parametrize("T", [0.95, 1.2])
def test_shear_viscosity_is_theta_times_tau(T):
    # Chapman-Enskog with the exact third moment: nu = theta (tau_l - 1/2),
    # theta = T/s, i.e. eta = n T (tau - dt/2) in the paper's units (D2Q9 has
    # n (tau - dt/2) at every T). The discrete rate approaches nu k^2 with an
    # O(k^2) relative error: extrapolate from L = 64 and 128.
    tau = 0.6
    s = o17.lattice()[3]
    nu = T / s * (math.sqrt(s) * tau - 0.5)
    r64, r128 = _shear_rate(17, 64, T, tau), _shear_rate(17, 128, T, tau, steps=1200)
    k64, k128 = 2 * math.pi / 64, 2 * math.pi / 128
    assert abs(r128 / (nu * k128 ** 2) - 1) < 2e-3
    extrap = (4 * r128 / k128 ** 2 - r64 / k64 ** 2) / 3
    assert abs(extrap / nu - 1) < 2e-4


def test_viscosity_is_galilean_invariant_unlike_d2q9():
    # The u*^3 term: D2Q9 misses n u_x u_x u_y in the third moment, so a shear
    # wave carried by a flow U along its wave vector decays with
    # (1/3 - U^2)(tau_l - 1/2) instead of (tau_l - 1/2)/3. D2Q17 carries that
    # moment and its rate does not depend on U.
    T, tau = 0.95, 0.6
    base17, base9 = _shear_rate(17, 64, T, tau), _shear_rate(9, 64, T, tau)
    for U in (0.05, 0.1):
        r17 = _shear_rate(17, 64, T, tau, U=U)
        r9 = _shear_rate(9, 64, T, tau, U=U)
        assert abs(r17 / base17 - 1) < 1e-4
        assert abs(r9 / base9 - (1 - 3 * U * U)) < 5e-4
        assert r9 / base9 < 1 - 2 * U * U


def _quench(T=0.9, V0=0.01, L=(96, 64), seed=5):
    w = ls.Workload("d2q17", L[0], L[1], T=T, V0=V0, k=2, y_periodic=True, seed=seed)
    p = Params(w.Lx, w.Ly, T=T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, y_periodic=True)
    return w, p


def test_mass_is_conserved_and_the_rest_state_is_stationary():
    w, p = _quench()
    o = o17.Oracle17(p, w.n0(), fext=w.fext())
    m0 = o.mass()
    o.run(300)
    assert np.isfinite(o.S).all()
    assert abs(o.mass() / m0 - 1) < 1e-13
    assert o.n.max() - o.n.min() > 0.3          # the quench separates phases
    r = o17.Oracle17(p, np.full((p.Ly, p.Lx), 0.7))
    S0 = r.S.copy()
    r.run(50)
    assert np.abs(r.S - S0).max() < 1e-14


def test_transpose_and_mirror_symmetry():
    g = np.random.default_rng(3)
    L = 24
    p = Params(L, L, T=0.95, tau=0.8, kappa=0.3, N=0.3, Q=2.0, y_periodic=True)
    n0 = 0.7 + 0.05 * g.standard_normal((L, L))
    a = o17.Oracle17(p, n0)
    b = o17.Oracle17(p, np.ascontiguousarray(n0.T))
    c = o17.Oracle17(p, np.ascontiguousarray(n0[:, ::-1]))
    for o in (a, b, c):
        o.run(40)
    assert np.abs(b.n - a.n.T).max() < 1e-12
    assert np.abs(b.uy - a.ux.T).max() < 1e-12
    assert np.abs(c.n - a.n[:, ::-1]).max() < 1e-12
    assert np.abs(c.ux + a.ux[:, ::-1]).max() < 1e-12


def test_flat_interface_has_the_d2q9_coexistence_densities():
    # the velocity set does not enter the model's thermodynamics (force and
    # ideal pressure are the same): a relaxed planar interface has D2Q9's
    # bulk densities to within the lattices' discretisation differences, both
    # about 1e-2 from the Maxwell construction
    T, L = 0.95, 96
    nl, nv, _ = cf.maxwell(T)
    p = Params(L, 4, T=T, tau=1.0, N=0.3, Q=2.0, y_periodic=True)
    n0 = ls.flat_interface(L, 4, nv, nl, axis="x")
    a, b = OracleLB(p, n0), o17.Oracle17(p, n0)
    a.run(24000)
    b.run(24000)
    assert abs(b.n[0, 48] - a.n[0, 48]) < 5e-4 and abs(b.n[0, 0] - a.n[0, 0]) < 5e-4
    assert abs(b.n[0, 48] - nl) < 1.2e-2 and abs(b.n[0, 0] - nv) < 2e-2
    assert np.abs(b.ux).max() < 1e-4


def test_rejects_walls_and_regularised_collision():
    with pytest.raises(ValueError):
        o17.Oracle17(Params(8, 8, y_periodic=False), np.ones((8, 8)))
    with pytest.raises(ValueError):
        o17.Oracle17(Params(8, 8, y_periodic=True, regularized=True), np.ones((8, 8)))


def test_window_runs_are_exact_inside_the_dependency_cone():
    """A node's populations after a step depend on the stored populations at
    most 5 nodes away (pull reach 3, force stencils 2): a periodic window run
    from the same initial fields equals the full run bitwise on nodes farther
    than 5 S from the window's edges after S steps. (Used by the full-size GPU
    test to check 8192 x 2048.)"""
    w, p = _quench(L=(96, 80))
    n0, fext = w.n0(), w.fext()
    x0, y0, wx, wy = 30, 20, 50, 46
    pw = Params(wx, wy, T=p.T, tau=p.tau, kappa=p.kappa, N=p.N, Q=p.Q, y_periodic=True)
    sub = (slice(None), slice(y0, y0 + wy), slice(x0, x0 + wx))
    for S in (1, 4):
        full = o17.Oracle17(p, n0, fext=fext)
        full.run(S)
        win = o17.Oracle17(pw, np.ascontiguousarray(n0[y0:y0 + wy, x0:x0 + wx]),
                           fext=fext[x0:x0 + wx])
        win.run(S)
        m = 5 * S
        inner = (slice(None), slice(m, wy - m), slice(m, wx - m))
        assert np.array_equal(win.S[inner], full.S[sub][inner])
        if S == 1:
            # one node closer to the edge is already different: the cone is
            # tight (after more steps the difference at its rim falls below
            # rounding)
            edge = (slice(None), slice(m - 1, wy - m + 1), slice(m - 1, wx - m + 1))
            assert not np.array_equal(win.S[edge], full.S[sub][edge])
