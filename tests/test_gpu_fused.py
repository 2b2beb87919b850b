"""The two-step kernel (lb_set_launch_fused) against the one-step kernel and
the oracle.

Every node of the two-step kernel runs the arithmetic of two single steps
on the same inputs, with mirror reads at the walls standing in for the
one-step kernel's ghost rows, so populations and moments must agree bit for
bit with one step per launch: walls and periodic y, ragged strips and
chunks, chunks that start within three rows of a wall, both march
directions, odd step counts, checks that split pairs, the drift shift, and
the moments written by the last launch."""
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


def _lattice(Lx, Ly, periodic, seed, check_every=0, drift=False, U=0.03, V0=0.1, k=2, T=0.95,
             tau=1.0, regularized=False):
    from paper_1307_6703_amd import Lattice
    N, Q = ls.table1_nq(T)
    g = Lattice(Lx, Ly, T=T, tau=tau, kappa=0.3, N=N, Q=Q, U=0.0 if periodic else U,
                fext=ls.potential_force(Lx, V0, k), y_periodic=periodic, fp32=True,
                check_every=check_every, drift_correct=drift, regularized=regularized)
    g.init(ls.noisy_density(Lx, Ly, seed))
    return g


CASES = [
    # Lx, Ly, periodic, (threads, rows), steps
    (300, 70, False, (128, 8), 41),
    (300, 70, True, (128, 9), 40),
    (300, 70, False, (192, 17), 40),
    (300, 70, False, (256, 70), 40),
    (129, 37, False, (128, 33), 23),     # chunk of 4 rows at the upper wall
    (100, 4, False, (128, 8), 20),       # smallest Ly: one chunk between two walls
    (100, 5, True, (128, 8), 21),
    (57, 12, False, (256, 8), 30),       # one strip wider than the lattice
    (514, 40, True, (192, 8), 12),
    (1, 9, False, (128, 8), 14),         # one column: every pull wraps onto itself
    (2, 6, True, (128, 8), 9),
    (115, 33, False, (128, 1), 10),      # chunks of 8 rows (the minimum), one column past a strip
    (300, 70, False, (64, 8), 41),       # one-wave workgroups: strips of 50 columns
    (101, 37, True, (64, 17), 20),       # one column past two strips
    (3, 9, False, (64, 8), 14),
    # 256-thread strips with walls: chunks whose pipeline stays at least one
    # row inside the walls run the wall-free body (the first such chunk
    # starts at row 8), the chunks at the walls the general one; the rows the
    # last chunk would lack come off the first and the last chunk
    (600, 64, False, (256, 8), 30),
    (600, 100, False, (256, 24), 41),
    (600, 96, False, (256, 16), 40),
    (600, 40, True, (256, 16), 20),
]


@pytest.mark.parametrize("Lx,Ly,periodic,launch,steps", CASES)
def test_fused_equals_one_step_bitwise(torch_cuda, Lx, Ly, periodic, launch, steps):
    _say("fused vs one-step", Lx, Ly, periodic, launch, steps)
    a = _lattice(Lx, Ly, periodic, seed=Lx + 7 * Ly)
    b = _lattice(Lx, Ly, periodic, seed=Lx + 7 * Ly)
    b.set_launch(*launch, steps_per_launch=2)
    assert b.steps_per_launch() == 2
    a.step(steps)
    b.step(steps)
    assert a.step_count == b.step_count == steps
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.populations(), b.populations())


# the regularised collision (Sec. II's re-projection) in both kernels, at
# tau = 1 and at tau = 2 where the projection changes most
REG_CASES = [
    (300, 70, False, (128, 8), 41, 2.0),
    (300, 70, True, (128, 9), 40, 2.0),
    (600, 100, False, (256, 24), 41, 1.0),
    (600, 40, True, (256, 16), 20, 2.0),
    (101, 37, True, (64, 17), 20, 2.0),
    (1, 9, False, (128, 8), 14, 1.0),
]


@pytest.mark.parametrize("Lx,Ly,periodic,launch,steps,tau", REG_CASES)
def test_regularised_fused_equals_one_step_bitwise(torch_cuda, Lx, Ly, periodic, launch, steps,
                                                   tau):
    _say("regularised fused vs one-step", Lx, Ly, periodic, launch, steps, tau)
    a = _lattice(Lx, Ly, periodic, seed=Lx + 5 * Ly, tau=tau, regularized=True)
    b = _lattice(Lx, Ly, periodic, seed=Lx + 5 * Ly, tau=tau, regularized=True)
    b.set_launch(*launch, steps_per_launch=2)
    assert b.steps_per_launch() == 2
    a.step(steps)
    b.step(steps)
    for x, y in zip(a.moments(), b.moments()):
        assert np.array_equal(x, y)
    assert np.array_equal(a.populations(), b.populations())


def test_regularised_fused_matches_oracle(torch_cuda):
    w = ls.PARITY_FP64
    _say("regularised fused fp32 vs oracle", w.name)
    N, Q = ls.table1_nq(w.T)
    from paper_1307_6703_amd import Lattice
    fext = ls.potential_force(w.Lx, w.V0, w.k)
    n0 = ls.noisy_density(w.Lx, w.Ly, w.seed)
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=2.0, kappa=0.3, N=N, Q=Q, U=w.U, fext=fext, fp32=True,
                check_every=100, drift_correct=True, regularized=True)
    g.set_launch(128, 0, steps_per_launch=2)
    g.init(n0)
    o = OracleLB(Params(w.Lx, w.Ly, T=w.T, tau=2.0, kappa=0.3, N=N, Q=Q, U=w.U,
                        regularized=True), n0, fext=fext)
    g.step(200)
    o.run(200, threads=8)
    n, ux, uy = g.moments()
    rel = (np.abs(n - o.n) / o.n).max()
    du = max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max())
    _say(f"max rel |dn| {rel:.2e}, max |du| {du:.2e}")
    assert rel <= 1e-4 and du <= 1e-4


def test_fused_with_checks_and_drift_shift(torch_cuda):
    # check_every = 7: pairs never straddle a check, so single steps appear
    # before every check; the drift shift is applied by whichever kernel
    # takes the next step
    _say("fused with checks every 7 and drift correction")
    a = _lattice(260, 48, False, seed=5, check_every=7, drift=True)
    b = _lattice(260, 48, False, seed=5, check_every=7, drift=True)
    b.set_launch(128, 17, steps_per_launch=2)
    for n in (1, 6, 13, 30):
        a.step(n)
        b.step(n)
        assert np.array_equal(a.populations(), b.populations()), n
        for x, y in zip(a.moments(), b.moments()):
            assert np.array_equal(x, y)
    ra, rb = a.reduce(), b.reduce()
    assert ra == rb


def test_fused_matches_oracle(torch_cuda):
    w = ls.PARITY_FP64
    _say("fused fp32 vs oracle", w.name)
    N, Q = ls.table1_nq(w.T)
    from paper_1307_6703_amd import Lattice
    fext = ls.potential_force(w.Lx, w.V0, w.k)
    n0 = ls.noisy_density(w.Lx, w.Ly, w.seed)
    g = Lattice(w.Lx, w.Ly, T=w.T, tau=1.0, kappa=0.3, N=N, Q=Q, U=w.U, fext=fext, fp32=True,
                check_every=100, drift_correct=True)
    g.set_launch(128, 0, steps_per_launch=2)
    g.init(n0)
    o = OracleLB(Params(w.Lx, w.Ly, T=w.T, tau=1.0, kappa=0.3, N=N, Q=Q, U=w.U), n0, fext=fext)
    g.step(200)
    o.run(200, threads=8)
    n, ux, uy = g.moments()
    rel = (np.abs(n - o.n) / o.n).max()
    du = max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max())
    _say(f"max rel |dn| {rel:.2e}, max |du| {du:.2e}")
    assert rel <= 1e-4 and du <= 1e-4


def test_fused_launch_is_validated(torch_cuda):
    from paper_1307_6703_amd import Lattice, LBError
    g = Lattice(64, 16, fp32=False)
    with pytest.raises(LBError):
        g.set_launch(128, 0, steps_per_launch=2)  # FP64 storage
    g.close()
    g = Lattice(64, 16, fp32="sr")
    with pytest.raises(LBError):
        g.set_launch(128, 0, steps_per_launch=2)  # FP64 arithmetic, stochastic rounding
    with pytest.raises(LBError):
        g.set_launch(512, 0)  # 512-thread strips: FP32 arithmetic only
    g.close()
    g = _lattice(64, 16, False, seed=1)
    for t in (96, 320, 512):
        with pytest.raises(LBError):
            g.set_launch(t, 0, steps_per_launch=2)
    g.set_launch(0, 0, steps_per_launch=2)
    assert g.steps_per_launch() == 2 and g.get_launch()[0] == 128
    g.set_launch(0, 0)
    assert g.steps_per_launch() == 1


def _batch_instances():
    out = []
    for i, w in enumerate(ls.batch_draws(7, seed=23)):
        Lx, Ly = w.Lx // 2 + 5 * i, w.Ly // 2 + 3 * i  # uneven and ragged
        out.append(dict(Lx=Lx, Ly=Ly, T=w.T, U=w.U, N=w.N, Q=w.Q, tau=w.tau, kappa=w.kappa,
                        fext=ls.potential_force(Lx, w.V0, w.k), y_periodic=(i % 3 == 2),
                        seed=w.seed))
    return out


@pytest.mark.parametrize("check_every,launch,reg", [(20, (128, 33), False), (7, (256, 17), False),
                                                    (0, (192, 65), False), (20, (64, 40), False),
                                                    (7, (128, 24), True)])
def test_batch_fused_equals_one_step_batch(torch_cuda, check_every, launch, reg):
    # graph runs of 64 steps (32 launches), eager steps up to the check grid,
    # single steps before checks that split a pair, subset steps
    from paper_1307_6703_amd import Batch
    _say("batch fused vs one-step", check_every, launch, reg)
    insts = _batch_instances()
    specs = [{k: v for k, v in d.items() if k != "seed"} for d in insts]
    drift = check_every > 0
    a = Batch(specs, fp32=True, check_every=check_every, drift_correct=drift, regularized=reg)
    b = Batch(specs, fp32=True, check_every=check_every, drift_correct=drift, regularized=reg)
    for i, d in enumerate(insts):
        a.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
        b.init(i, ls.noisy_density(d["Lx"], d["Ly"], d["seed"]))
    b.set_launch(*launch, steps_per_launch=2)
    assert b.steps_per_launch() == 2
    for n in (151, 6, 77):
        a.step(n)
        b.step(n)
        for i in range(len(insts)):
            for x, y in zip(a.moments(i), b.moments(i)):
                assert np.array_equal(x, y), (n, i)
    mask = [1 if i % 2 else 0 for i in range(len(insts))]
    for n in (10, 8, 2):  # 4 pairs + 2 single steps, 4 pairs, 2 single steps
        a.step_subset(n, mask)
        b.step_subset(n, mask)
    a.step(3)
    b.step(3)
    for i in range(len(insts)):
        for x, y in zip(a.moments(i), b.moments(i)):
            assert np.array_equal(x, y), ("subset", i)
    assert all(s == 0 for s in b.status())


def test_default_shape(torch_cuda):
    from paper_1307_6703_amd import Lattice
    # 256-thread strips (242 columns) when they cover Lx with at most 3% to
    # spare, else 128: 2048 needs 9 x 242 = 2178 (6% over), 8192 34 x 242
    # = 8228 (0.4%), 4096 17 x 242 = 4114 (0.4%)
    for Lx, Ly, th in ((2048, 512, 128), (8192, 128, 256), (4096, 256, 256)):
        big = Lattice(Lx, Ly, fp32=True)
        assert big.steps_per_launch() == 2 and big.get_launch()[0] == th, (Lx, Ly, big.get_launch())
        big.close()
    for kw in (dict(Lx=2048, Ly=512, fp32=False), dict(Lx=300, Ly=70, fp32=True),
               dict(Lx=128, Ly=8192, fp32=True)):
        g = Lattice(kw.pop("Lx"), kw.pop("Ly"), **kw)
        assert g.steps_per_launch() == 1, kw
        g.close()
