"""The batched path: many uneven lattices in one launch per step, replayed
from a HIP graph. Each instance must equal its single-lattice run bitwise
(the per-node arithmetic does not depend on which launch runs it), and a
subset must match the oracle."""
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
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _instances(fp32):
    out = []
    for i, w in enumerate(ls.batch_draws(7, seed=11)):
        Lx, Ly = w.Lx // 4 + 3 * i, w.Ly // 4 + i  # small and ragged
        out.append(dict(Lx=Lx, Ly=Ly, T=w.T, U=w.U, N=w.N, Q=w.Q, tau=w.tau, kappa=w.kappa,
                        fext=ls.potential_force(Lx, w.V0, w.k), y_periodic=(i % 3 == 2),
                        seed=w.seed))
    return out


def _single(inst, fp32, steps, check_every=0, drift=False, launch=None):
    from paper_1307_6703_amd import Lattice
    kw = dict(inst)
    seed = kw.pop("seed")
    g = Lattice(kw.pop("Lx"), kw.pop("Ly"), fp32=fp32, check_every=check_every,
                drift_correct=drift, **kw)
    if launch:
        g.set_launch(*launch)
    g.init(ls.noisy_density(g.Lx, g.Ly, seed))
    g.step(steps)
    return g


@pytest.mark.parametrize("fp32", [True, False, "sr"])
def test_batch_equals_single_runs_bitwise(torch_cuda, fp32):
    from paper_1307_6703_amd import Batch
    _say("batch vs single", "fp32" if fp32 else "fp64")
    insts = _instances(fp32)
    b = Batch([{k: v for k, v in d.items() if k != "seed"} for d in insts], fp32=fp32,
              check_every=20, drift_correct=bool(fp32))
    for i, d in enumerate(insts):
        b.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
    steps = 150  # graph runs of 64 steps, checks every 20, eager tail
    b.step(steps)
    for i, d in enumerate(insts):
        g = _single(d, fp32, steps, check_every=20, drift=bool(fp32))
        nb, uxb, uyb = b.moments(i)
        n, ux, uy = g.moments()
        assert np.array_equal(nb, n) and np.array_equal(uxb, ux) and np.array_equal(uyb, uy), i
    assert all(s == 0 for s in b.status())


def test_batch_subset_matches_oracle(torch_cuda):
    from paper_1307_6703_amd import Batch
    _say("batch vs oracle")
    insts = _instances(False)[:3]
    b = Batch([{k: v for k, v in d.items() if k != "seed"} for d in insts], fp32=False)
    for i, d in enumerate(insts):
        b.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
    b.step(130)
    for i, d in enumerate(insts):
        o = OracleLB(Params(d["Lx"], d["Ly"], T=d["T"], tau=d["tau"], kappa=d["kappa"], N=d["N"],
                            Q=d["Q"], U=d["U"], y_periodic=d["y_periodic"]),
                     ls.noisy_density(d["Lx"], d["Ly"], d["seed"]), fext=d["fext"])
        o.run(130, threads=8)
        n, ux, uy = b.moments(i)
        assert np.abs(n - o.n).max() <= 1e-10
        assert max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max()) <= 1e-10


def test_batch_reports_unstable_instances(torch_cuda):
    from paper_1307_6703_amd import Batch, LBError, lbvdw
    _say("batch status")
    good = dict(Lx=40, Ly=20, T=0.95, U=0.01)
    bad = dict(Lx=40, Ly=20, T=0.5, y_periodic=True)
    b = Batch([good, bad], fp32=True, check_every=10)
    b.init(0, ls.noisy_density(40, 20, 1))
    b.init(1, ls.noisy_density(40, 20, 2, amp=0.2))
    b.step(300)
    st = b.status()
    assert st[0] == lbvdw.LB_OK and st[1] == lbvdw.LB_EUNSTABLE
    with pytest.raises(LBError):
        b.step(1)
    # dropping the unstable instance lets the other one go on, unchanged by
    # its neighbour: it equals a batch that never held the unstable one
    assert b.drop_unstable() == 1
    b.step(200)
    assert b.status() == [lbvdw.LB_OK, lbvdw.LB_EUNSTABLE]
    c = Batch([good], fp32=True, check_every=10)
    c.init(0, ls.noisy_density(40, 20, 1))
    c.step(500)
    for u, v in zip(b.moments(0), c.moments(0)):
        assert np.array_equal(u, v)
    with pytest.raises(LBError):
        b.moments(1)


def test_batch_autotune_keeps_results(torch_cuda):
    from paper_1307_6703_amd import Batch
    _say("batch autotune")
    insts = _instances(True)
    specs = [{k: v for k, v in d.items() if k != "seed"} for d in insts]
    a = Batch(specs, fp32=True)
    c = Batch(specs, fp32=True)
    for i, d in enumerate(insts):
        a.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
        c.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
    t, r, ms = a.autotune(nsteps=2)
    assert t in (64, 128, 192, 256, 512) and ms > 0
    # autotune took 15 one-step shapes x (1 + 2) steps and 24 two-step shapes
    # x (2 + 2) steps
    c.step(15 * 3 + 24 * 4)
    a.step(1)
    c.step(1)
    for i in range(len(insts)):
        assert np.array_equal(a.moments(i)[0], c.moments(i)[0])
