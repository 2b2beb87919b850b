"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 8192 x 2048 sheared lattice, FP32 and FP64, 3 steps against the
oracle on every node, and 100 steps on columns where an oracle run on a
window of the lattice is exact."""
import sys

import numpy as np
import pytest

import lbsynth as ls
from oracle.lb_oracle import OracleLB, Params

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    w = ls.ROOFLINE
    n0, fext = w.n0(), w.fext()
    o = OracleLB(Params(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U),
                 n0, fext=fext)
    _say("oracle full size, 3 steps")
    o.run(3)
    return w, n0, fext, o


def _key(w, fp32):
    return f"{w.Lx}x{w.Ly}-{ {True: 'fp32', False: 'fp64', 'sr': 'fp32sr'}[fp32]}-gfx950"


@pytest.mark.parametrize("fp32,tol", [(True, 1e-4), (False, 1e-10), ("sr", 1e-4)])
def test_full_size_parity(setup, fp32, tol):
    import bench
    from paper_1307_6703_amd import Lattice
    w, n0, fext, o = setup
    _say("full size", w.name, fp32)
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                fp32=fp32, check_every=100, drift_correct=bool(fp32))
    launch = bench.tuned_launch(_key(w, fp32))
    if launch:
        g.set_launch(*launch)
    g.init(n0).step(3)
    n, ux, uy = g.moments()
    rel = np.abs(n - o.n) / o.n
    du = max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max())
    _say(f"launch {g.get_launch()}: max rel |dn| {rel.max():.2e}, max |du| {du:.2e}")
    if fp32:
        assert rel.max() <= tol and du <= tol
    else:
        assert np.abs(n - o.n).max() <= tol and du <= tol
    g.close()


# One step reaches 4 columns (pulls +-1, then the density stencils +-3), so
# after S steps a node depends only on columns within 4 S of it. An oracle run
# on a window of the full lattice, periodic at its cut edges, is therefore
# exact (to rounding) on the columns farther than 4 S from those edges.
WINDOW_STEPS = 100
WINDOW_HALF = 4 * WINDOW_STEPS + 50
WINDOW_KEEP = 48


_WINDOWS = {}


def _oracle_window(w, n0, fext, x0):
    if x0 not in _WINDOWS:
        cols = np.arange(x0 - WINDOW_HALF, x0 + WINDOW_HALF) % w.Lx
        _say(f"oracle window of {cols.size} columns at x0 = {x0}, {WINDOW_STEPS} steps")
        o = OracleLB(Params(cols.size, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U),
                     np.ascontiguousarray(n0[:, cols]), fext=np.ascontiguousarray(fext[cols]))
        o.run(WINDOW_STEPS)
        _WINDOWS[x0] = (cols, o)
    return _WINDOWS[x0]


@pytest.mark.parametrize("x0", [4000, 20])   # an interior window and one across x = 0
@pytest.mark.parametrize("fp32,tol", [(True, 1e-4), (False, 1e-10), ("sr", 1e-4)])
def test_full_size_100_steps_on_exact_windows(fp32, tol, x0):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    from paper_1307_6703_amd import Lattice
    w = ls.ROOFLINE
    n0, fext = w.n0(), w.fext()
    cols, o = _oracle_window(w, n0, fext, x0)
    _say("full size", w.name, fp32, WINDOW_STEPS, "steps")
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                fp32=fp32, check_every=100, drift_correct=bool(fp32))
    launch = bench.tuned_launch(_key(w, fp32))
    if launch:
        g.set_launch(*launch)
    g.init(n0).step(WINDOW_STEPS)
    n, ux, uy = g.moments()
    g.close()
    keep = slice(WINDOW_HALF - WINDOW_KEEP, WINDOW_HALF + WINDOW_KEEP)
    gx = cols[keep]
    on, oux, ouy = o.n[:, keep], o.ux[:, keep], o.uy[:, keep]
    rel = np.abs(n[:, gx] - on) / on
    du = max(np.abs(ux[:, gx] - oux).max(), np.abs(uy[:, gx] - ouy).max())
    _say(f"columns {gx[0]}..{gx[-1]}: max rel |dn| {rel.max():.2e}, max |du| {du:.2e}")
    if fp32:
        assert rel.max() <= tol and du <= tol
    else:
        assert np.abs(n[:, gx] - on).max() <= tol and du <= tol


_REG_WINDOWS = {}


@pytest.mark.parametrize("x0", [4000])
def test_full_size_regularised_two_step_on_exact_window(x0):
    """The regularised collision on the full lattice in its default launch
    (two steps per launch in FP32), 100 steps at tau = 2 (at tau = 1 the
    projection has no effect), against an exact oracle window."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_6703_amd import Lattice
    w = ls.ROOFLINE
    tau = 2.0
    n0, fext = w.n0(), w.fext()
    if x0 not in _REG_WINDOWS:
        cols = np.arange(x0 - WINDOW_HALF, x0 + WINDOW_HALF) % w.Lx
        _say(f"regularised oracle window of {cols.size} columns at x0 = {x0}, {WINDOW_STEPS} steps")
        o = OracleLB(Params(cols.size, w.Ly, T=w.T, tau=tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                            regularized=True),
                     np.ascontiguousarray(n0[:, cols]), fext=np.ascontiguousarray(fext[cols]))
        o.run(WINDOW_STEPS)
        _REG_WINDOWS[x0] = (cols, o)
    cols, o = _REG_WINDOWS[x0]
    _say("full size regularised", w.name, WINDOW_STEPS, "steps")
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                fp32=True, check_every=100, drift_correct=True, regularized=True)
    assert g.steps_per_launch() == 2
    g.init(n0).step(WINDOW_STEPS)
    n, ux, uy = g.moments()
    _say(f"launch {g.get_launch()}")
    g.close()
    keep = slice(WINDOW_HALF - WINDOW_KEEP, WINDOW_HALF + WINDOW_KEEP)
    gx = cols[keep]
    on, oux, ouy = o.n[:, keep], o.ux[:, keep], o.uy[:, keep]
    rel = np.abs(n[:, gx] - on) / on
    du = max(np.abs(ux[:, gx] - oux).max(), np.abs(uy[:, gx] - ouy).max())
    _say(f"columns {gx[0]}..{gx[-1]}: max rel |dn| {rel.max():.2e}, max |du| {du:.2e}")
    assert rel.max() <= 1e-4 and du <= 1e-4
