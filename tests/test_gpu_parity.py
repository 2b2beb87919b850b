"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

FP64 mode: every density and velocity within 1e-10 (absolute). FP32 storage
(FP32 arithmetic, or FP64 arithmetic with stochastic rounding of the stored
values, "sr"): within 1e-4 relative to the density. Inputs are seeded and identical on both
sides (lbsynth). Each case prints its name first, so a failing GPU run names
the case that was running."""
import math
import sys

import numpy as np
import pytest

import lbsynth as ls
from oracle.lb_oracle import OracleLB, Params

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pair(Lx, Ly, *, T=0.95, tau=1.0, kappa=0.3, N=None, Q=None, U=0.0, V0=0.0, k=1,
          periodic=False, fp32=False, seed=1307, n0=None, launch=None, regularized=False,
          **extra):
    from paper_1307_6703_amd import Lattice
    if N is None or Q is None:
        N, Q = ls.table1_nq(T)
    fext = ls.potential_force(Lx, V0, k)
    if n0 is None:
        n0 = ls.noisy_density(Lx, Ly, seed)
    g = Lattice(Lx, Ly, T=T, tau=tau, kappa=kappa, N=N, Q=Q, U=U, fext=fext,
                y_periodic=periodic, fp32=fp32, regularized=regularized, **extra)
    if launch:
        g.set_launch(*launch)
    g.init(n0)
    o = OracleLB(Params(Lx, Ly, T=T, tau=tau, kappa=kappa, N=N, Q=Q, U=U, y_periodic=periodic,
                        regularized=regularized), n0, fext=fext)
    return g, o


def _cmp(g, o):
    n, ux, uy = g.moments()
    return (np.abs(n - o.n).max(), np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max(),
            (np.abs(n - o.n) / o.n).max())


def test_fp64_parity_sheared_zebra_128x64(torch_cuda):
    # The FP64 parity workload: 128 x 64 between walls at +-0.01, T = 0.95,
    # V(x) = 0.05 sin(2 pi 4 x / 128), seeded noise, 2000 steps.
    w = ls.PARITY_FP64
    _say("fp64", w.name)
    g, o = _pair(w.Lx, w.Ly, T=w.T, U=w.U, V0=w.V0, k=w.k, seed=w.seed)
    m0 = g.reduce()["mass"]
    done = 0
    for upto in (1, 10, 100, 500, 2000):
        g.step(upto - done)
        o.run(upto - done, threads=8)
        done = upto
        dn, dux, duy, _ = _cmp(g, o)
        _say(f"step {upto}: |dn| {dn:.2e} |dux| {dux:.2e} |duy| {duy:.2e}")
        assert dn <= TOL64 and dux <= TOL64 and duy <= TOL64
    m = g.reduce()["mass"]
    assert abs(m - m0) / m0 <= 1e-13
    assert abs(m - o.mass()) / m0 <= 1e-13


def test_fp64_parity_periodic_droplet(torch_cuda):
    _say("fp64 periodic droplet 96x40")
    T = 0.95
    n0 = ls.droplet(96, 40, 10.0, 1.46, 0.58) + 0.002 * ls.noisy_density(96, 40, 3, mean=0.0, amp=1.0)
    g, o = _pair(96, 40, T=T, periodic=True, n0=n0)
    g.step(300)
    o.run(300, threads=8)
    dn, dux, duy, _ = _cmp(g, o)
    assert dn <= TOL64 and dux <= TOL64 and duy <= TOL64


RAGGED = [
    # (Lx, Ly, periodic, launch)
    (1, 16, False, (64, 8)),
    (5, 7, True, (64, 8)),
    (7, 4, False, (128, 8)),
    (58, 9, False, (64, 8)),      # exactly one full 64-thread strip
    (59, 33, True, (64, 13)),     # one column over: a one-wide second strip
    (250, 12, False, (256, 8)),
    (251, 40, False, (256, 16)),
    (300, 21, True, (128, 10)),
    (513, 20, False, (256, 64)),
    (700, 30, True, (320, 10)),
]


@pytest.mark.parametrize("Lx,Ly,periodic,launch", RAGGED)
def test_fp64_parity_ragged_shapes(torch_cuda, Lx, Ly, periodic, launch):
    _say("fp64 ragged", Lx, Ly, periodic, launch)
    g, o = _pair(Lx, Ly, U=0.02, V0=0.1, k=1, periodic=periodic, seed=Lx * 1000 + Ly,
                 launch=launch)
    g.step(25)
    o.run(25, threads=8)
    dn, dux, duy, _ = _cmp(g, o)
    assert dn <= TOL64 and dux <= TOL64 and duy <= TOL64


@pytest.mark.parametrize("fp32", [False, True, "sr"])
def test_launch_shape_does_not_change_results(torch_cuda, fp32):
    # with stochastic rounding too: the draws depend on the node and the step,
    # not on which workgroup updates the node
    _say("launch shapes bitwise", fp32)
    Lx, Ly = 300, 70
    ref = None
    shapes = [(64, 8), (128, 16), (256, 70), (256, 9), (128, 64), (320, 18)]
    if fp32 is True:
        shapes.append((512, 26))
    for launch in shapes:
        g, _ = _pair(Lx, Ly, U=0.03, V0=0.1, k=3, fp32=fp32, launch=launch)
        g.step(40)
        f = g.populations()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f, ref), launch


@pytest.mark.parametrize("fp32", [True, "sr"])
def test_fp32_parity_short_horizon(torch_cuda, fp32):
    w = ls.PARITY_FP64
    _say("fp32 vs oracle", w.name, fp32)
    g, o = _pair(w.Lx, w.Ly, T=w.T, U=w.U, V0=w.V0, k=w.k, seed=w.seed, fp32=fp32)
    done = 0
    for upto in (1, 10, 100, 200):
        g.step(upto - done)
        o.run(upto - done, threads=8)
        done = upto
        _, dux, duy, rel = _cmp(g, o)
        _say(f"step {upto}: rel |dn| {rel:.2e} |du| {max(dux, duy):.2e}")
        assert rel <= TOL32
        assert max(dux, duy) <= TOL32


def test_wall_nodes_move_with_walls(torch_cuda):
    _say("wall velocities")
    U = 0.05
    g, _ = _pair(64, 32, U=U, V0=0.1, k=2)
    g.step(50)
    n, ux, uy = g.moments()
    assert np.allclose(ux[0], -U, atol=1e-15) and np.allclose(ux[-1], U, atol=1e-15)
    assert np.abs(uy[[0, -1]]).max() <= 1e-15


def test_checkpoint_resume(torch_cuda):
    _say("checkpoint fp64")
    a, _ = _pair(130, 24, U=0.02, V0=0.05, k=2)
    b, _ = _pair(130, 24, U=0.02, V0=0.05, k=2)
    a.step(60)
    b.step(30)
    f = b.populations()
    b.set_populations(f, step=30)
    assert b.step_count == 30
    b.step(30)
    assert np.array_equal(a.populations(), b.populations())
    assert np.array_equal(a.moments()[0], b.moments()[0])


@pytest.mark.parametrize("fp32", [True, "sr"])
def test_checkpoint_resume_fp32(torch_cuda, fp32):
    _say("checkpoint fp32", fp32)
    a, _ = _pair(130, 24, U=0.02, V0=0.05, k=2, fp32=fp32)
    b, _ = _pair(130, 24, U=0.02, V0=0.05, k=2, fp32=fp32)
    a.step(60)
    b.step(30)
    b.set_populations(b.populations(), step=30)
    b.step(30)
    # the FP32 reference density is re-derived from the restored mass
    assert np.abs(a.moments()[0] - b.moments()[0]).max() <= 1e-6


@pytest.mark.parametrize("fp32", [True, "sr"])
def test_runs_are_deterministic(torch_cuda, fp32):
    _say("determinism", fp32)
    outs = []
    for _ in range(2):
        g, _ = _pair(200, 48, U=0.04, V0=0.1, k=4, fp32=fp32, check_every=7)
        g.step(77)
        outs.append((g.populations(), g.reduce()))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert outs[0][1] == outs[1][1]


def test_fp64_mass_is_conserved_on_gpu(torch_cuda):
    _say("fp64 mass")
    g, _ = _pair(256, 64, U=0.05, V0=0.1, k=4)
    m0 = g.reduce()["mass"]
    g.step(1000)
    r = g.reduce()
    assert abs(r["mass"] - m0) / m0 <= 1e-13
    assert r["nonfinite"] == 0 and 0 < r["nmin"] < r["nmax"] < 3


def test_fp32_drift_correction_holds_mass(torch_cuda):
    _say("fp32 drift")
    res = {}
    for drift in (False, True):
        g, _ = _pair(512, 128, T=0.95, U=0.05, V0=0.01, k=4, fp32=True, check_every=50,
                     drift_correct=drift)
        m0 = g.reduce()["mass"]
        g.step(5000)
        res[drift] = abs(g.reduce()["mass"] - m0) / m0
    _say("mass drift without / with correction", res[False], res[True])
    assert res[True] <= 1e-6
    assert res[True] <= res[False] + 1e-12


def test_instability_is_flagged(torch_cuda):
    _say("instability flag")
    from paper_1307_6703_amd import LBError, lbvdw
    # far below the temperatures the scheme handles: the liquid branch's sound
    # speed exceeds the lattice speed and the state leaves (0, 3)
    n0 = ls.noisy_density(64, 32, 5, amp=0.2)
    g, _ = _pair(64, 32, T=0.5, kappa=0.3, periodic=True, n0=n0, check_every=10)
    g.step(3000)
    with pytest.raises(LBError) as e:
        g.moments()
    assert e.value.status == lbvdw.LB_EUNSTABLE
    with pytest.raises(LBError) as e:
        g.step(1)
    assert e.value.status == lbvdw.LB_ESTATE


def test_invalid_initial_density_is_rejected(torch_cuda):
    _say("invalid n0")
    from paper_1307_6703_amd import LBError, Lattice, lbvdw
    g = Lattice(16, 8)
    bad = np.full((8, 16), 1.0)
    bad[3, 4] = 3.2
    with pytest.raises(LBError) as e:
        g.init(bad)
    assert e.value.status == lbvdw.LB_EINVAL
    with pytest.raises(LBError) as e:
        g.step(1)
    assert e.value.status == lbvdw.LB_ESTATE


def test_device_moments_match_host(torch_cuda):
    _say("device moments")
    g, _ = _pair(40, 20, U=0.01)
    g.step(5)
    d = g.moments_device().cpu().numpy()
    h = g.moments()
    for a, b in zip(d, h):
        assert np.array_equal(a, b)


def test_autotune_keeps_results(torch_cuda):
    _say("autotune")
    a, _ = _pair(600, 96, U=0.03, V0=0.1, k=2, fp32=True)
    b, _ = _pair(600, 96, U=0.03, V0=0.1, k=2, fp32=True)
    t, r, ms = a.autotune(nsteps=2)
    assert t in (64, 128, 192, 256, 512) and r >= 8 and ms > 0
    steps = a.step_count
    b.step(steps)
    assert np.array_equal(a.populations(), b.populations())


def test_stochastic_rounding_is_unbiased(torch_cuda):
    # A uniform flow in a periodic box: streaming leaves it unchanged and the
    # force, the gradients and D vanish, so one step is the collision
    # g' = (1 - omega) g + omega g_eq(n, u) of Eq.(evoleq) at every node, the
    # same at all of them. The host repeats it in FP64 from the stored state.
    # Rounding to nearest stores the same error at every node; stochastic
    # rounding stores the two neighbouring floats in proportions whose mean
    # is the exact value. Mean over 512 x 512 nodes of (stored - exact), in
    # float spacings: its standard error is below 1e-3.
    from paper_1307_6703_amd import Lattice
    _say("stochastic rounding bias")
    Lx = Ly = 512
    T, tau = 0.95, 1.0
    om = 1.0 / (math.sqrt(3.0) * tau)
    c = np.array([(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)], float)
    wts = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rest = wts * (1 + 0.5 * (T - 1) * (3 * (c ** 2).sum(1) - 2))
    worst = {True: 0.0, "sr": 0.0}
    for n0, ux0, uy0 in ((1.0, 0.0371, -0.0123), (0.7, 0.1, 0.05), (1.3, -0.02, 0.0)):
        for prec in (True, "sr"):
            g = Lattice(Lx, Ly, T=T, tau=tau, y_periodic=True, fp32=prec)
            g.init(np.full((Ly, Lx), n0), np.full((Ly, Lx), ux0), np.full((Ly, Lx), uy0))
            f0 = g.populations()
            nbar = n0  # the mean initial density
            gs = f0[:, 0, 0] - rest * nbar
            assert np.all(f0 == f0[:, :1, :1])  # uniform
            n = nbar + gs.sum()
            ux, uy = (c[:, 0] * gs).sum() / n, (c[:, 1] * gs).sum() / n
            cu = c[:, 0] * ux + c[:, 1] * uy
            geq = rest * (n - nbar) + wts * n * (3 * cu + 4.5 * cu * cu - 1.5 * (ux * ux + uy * uy))
            exact = (1 - om) * gs + om * geq
            g.step(1)
            f1 = g.populations()
            g.close()
            for i in range(9):
                ulp = float(np.spacing(np.float32(abs(exact[i]))))
                err = abs(float(np.mean(f1[i] - rest[i] * nbar)) - exact[i]) / ulp
                worst[prec] = max(worst[prec], err)
    _say(f"worst mean error in float spacings: nearest {worst[True]:.4f}, stochastic {worst['sr']:.5f}")
    assert worst["sr"] <= 0.01


# ---- regularised collision (the projection of f - f_eq onto the Hermite
# polynomials of order <= 2 before it relaxes) --------------------------------

@pytest.mark.parametrize("fp32,tol", [(False, TOL64), (True, TOL32), ("sr", TOL32)])
def test_regularised_parity_sheared_zebra_128x64(torch_cuda, fp32, tol):
    w = ls.PARITY_FP64
    _say("regularised", w.name, fp32)
    g, o = _pair(w.Lx, w.Ly, T=w.T, U=w.U, V0=w.V0, k=w.k, seed=w.seed, fp32=fp32,
                 regularized=True)
    done = 0
    for upto in (1, 10, 100, 500, 2000):
        g.step(upto - done)
        o.run(upto - done, threads=8)
        done = upto
        dn, dux, duy, rel = _cmp(g, o)
        _say(f"step {upto}: |dn| {dn:.2e} rel {rel:.2e} |du| {max(dux, duy):.2e}")
        if fp32 is False:
            assert dn <= tol and dux <= tol and duy <= tol
        else:
            assert rel <= tol and max(dux, duy) <= tol
    g.close()


@pytest.mark.parametrize("Lx,Ly,periodic,launch", [(59, 17, False, (64, 8)), (251, 9, True, (256, 4)),
                                                   (300, 33, False, (128, 10))])
def test_regularised_parity_ragged(torch_cuda, Lx, Ly, periodic, launch):
    _say("regularised ragged", Lx, Ly, periodic, launch)
    g, o = _pair(Lx, Ly, U=0.02, V0=0.1, k=1, periodic=periodic, seed=Lx + Ly, launch=launch,
                 tau=2.0, regularized=True)
    g.step(40)
    o.run(40, threads=8)
    dn, dux, duy, _ = _cmp(g, o)
    assert dn <= TOL64 and dux <= TOL64 and duy <= TOL64


def test_regularised_is_not_bgk_and_runs_two_steps_in_fp32_only(torch_cuda):
    from paper_1307_6703_amd import LBError
    _say("regularised vs bgk")
    a, _ = _pair(128, 32, U=0.03, V0=0.1, k=2, tau=2.0)
    b, _ = _pair(128, 32, U=0.03, V0=0.1, k=2, tau=2.0, regularized=True)
    a.step(50)
    b.step(50)
    assert np.abs(a.moments()[0] - b.moments()[0]).max() > 1e-8
    c, _ = _pair(300, 64, fp32=True, regularized=True)
    c.set_launch(128, 0, steps_per_launch=2)
    assert c.steps_per_launch() == 2
    d, _ = _pair(300, 64, fp32=False, regularized=True)
    with pytest.raises(LBError):
        d.set_launch(128, 0, steps_per_launch=2)
    for g in (a, b, c, d):
        g.close()
