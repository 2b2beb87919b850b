"""Parity at the benchmark's full size, in the launch configuration bench.py
times: the 8192 x 2048 sheared lattice, FP32 and FP64, a few steps against
the oracle on every node."""
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


@pytest.mark.parametrize("fp32,tol", [(True, 1e-4), (False, 1e-10)])
def test_full_size_parity(setup, fp32, tol):
    import bench
    from paper_1307_6703_amd import Lattice
    w, n0, fext, o = setup
    _say("full size", w.name, "fp32" if fp32 else "fp64")
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                fp32=fp32, check_every=100, drift_correct=fp32)
    launch = bench.tuned_launch(f"{w.Lx}x{w.Ly}-{'fp32' if fp32 else 'fp64'}-gfx950")
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
