"""The travelling interface wave under shear and a periodic force (Sec. IV,
Table 2) on the GPU path.

Setup as in the paper's second set of runs: T = 0.95, tau = 1, kappa = 0.3,
lambda = 32, walls at -+U with U = gamma_dot Ly / 2, gamma_dot = 1e-3 per
time step, Ly = 256, starting from a flat liquid-vapour interface along the
flow at Ly / 2 (Maxwell densities, tanh profile, seeded noise). The
amplitude A is the distance between the highest and lowest point of the
interface (the contour midway between the Maxwell densities).

What holds and is asserted: a single interface per column forms and carries
a stationary wave whose amplitude grows with Lx (512 -> 1024) and does not
depend on A0 (1e-4 vs 1e-5), as the paper reports. The absolute amplitude is
parity unpinned: the measured values are 0.5-0.75 of the printed ones
(printed beside them); the paper leaves the time and velocity units of
gamma_dot and tau open (readings c2 and c11)."""
import os
import sys

import numpy as np
import pytest

import lbsynth as ls
from oracle import closed_forms as cf

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

HERE = os.path.dirname(os.path.abspath(__file__))
LY, GDOT, STEPS, EVERY = 256, 1e-3, 300_000, 20_000


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _table2():
    rows = []
    for line in open(os.path.join(HERE, "golden", "table2_wave_amplitude.txt")):
        if line.strip() and not line.startswith("#"):
            T, lam, tau, g, A0, kap, Lx, Ly, A = line.split()
            rows.append((float(T), int(lam), float(tau), float(g), float(A0), float(kap), int(Lx),
                         int(Ly), float(A)))
    return rows


def _amplitude(n, T):
    nL, nV, _ = cf.maxwell(T)
    mid = 0.5 * (nL + nV)
    ys, single = [], 0
    for x in range(n.shape[1]):
        c = n[:, x] - mid
        s = np.nonzero(np.sign(c[:-1]) != np.sign(c[1:]))[0]
        if len(s) == 1:
            k = s[0]
            ys.append(k + c[k] / (c[k] - c[k + 1]))
            single += 1
    frac = single / n.shape[1]
    return ((max(ys) - min(ys)) / n.shape[0] if ys else float("nan")), frac


def test_interface_wave_amplitude_trends():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_6703_amd import Batch
    T, lam, tau, kap = 0.95, 32, 1.0, 0.3
    cases = [(512, 1e-4), (1024, 1e-4), (512, 1e-5), (1024, 1e-5)]
    N, Q = ls.table1_nq(T)
    nL, nV, _ = cf.maxwell(T)
    specs = [dict(Lx=Lx, Ly=LY, T=T, tau=tau, kappa=kap, N=N, Q=Q, U=GDOT * LY / 2,
                  fext=ls.sine_force(Lx, A0, lam)) for Lx, A0 in cases]
    b = Batch(specs, fp32=True, check_every=1000, drift_correct=True)
    y = np.arange(LY, dtype=np.float64)[:, None]
    prof = nV + (nL - nV) * 0.5 * (1.0 - np.tanh((y - LY / 2) / 2.0))
    for i, (Lx, _) in enumerate(cases):
        b.init(i, np.repeat(prof, Lx, axis=1) + (ls.noisy_density(Lx, LY, 2000 + i) - 1.0))
    b.autotune(nsteps=4)
    samples = {i: [] for i in range(len(cases))}
    done = 0
    while done < STEPS:
        b.step(EVERY)
        done += EVERY
        if done >= STEPS - 3 * EVERY:
            for i in range(len(cases)):
                samples[i].append(_amplitude(b.moments(i)[0], T))
        _say(f"step {done}")
    assert all(s == 0 for s in b.status())
    b.close()
    paper = {(r[6], r[4]): r[8] for r in _table2()
             if r[0] == T and r[1] == lam and r[2] == tau and r[5] == kap}
    A = {}
    for i, (Lx, A0) in enumerate(cases):
        amps = [a for a, f in samples[i]]
        fr = min(f for _, f in samples[i])
        A[(Lx, A0)] = float(np.mean(amps))
        print(f"Lx {Lx} A0 {A0:g}: A/Ly {A[(Lx, A0)]:.3f} (samples {np.round(amps, 3)}, "
              f"single-crossing columns {fr:.2f}); paper {paper.get((Lx, A0))}")
        assert fr == 1.0                                  # one interface in every column
        assert max(amps) - min(amps) <= 0.02              # stationary over the last 60k steps
    for A0 in (1e-4, 1e-5):
        assert A[(1024, A0)] >= A[(512, A0)] + 0.03       # grows with Lx
    for Lx in (512, 1024):
        assert abs(A[(Lx, 1e-4)] - A[(Lx, 1e-5)]) <= 0.03  # insensitive to A0


def _zebra_n0(Lx, seed):
    T = 0.95
    nL, nV, _ = cf.maxwell(T)
    y = np.arange(LY, dtype=np.float64)[:, None]
    prof = nV + (nL - nV) * 0.5 * (1.0 - np.tanh((y - LY / 2) / 2.0))
    return np.repeat(prof, Lx, axis=1) + (ls.noisy_density(Lx, LY, seed) - 1.0)


_ZEBRA_ORACLE = {}


@pytest.mark.parametrize("Lx", [1024, 2048])
@pytest.mark.parametrize("fp32,tol", [(False, 1e-10), (True, 1e-4), ("sr", 1e-4)])
def test_zebra_configuration_matches_oracle(Lx, fp32, tol):
    # The configuration of the runs above (literal sine force A0 sin(2 pi x /
    # lambda), walls at -+U, flat interface at Ly / 2 with noise), FP32 in
    # the two-step kernel, 100 steps against the oracle on every node.
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from oracle.lb_oracle import OracleLB, Params
    from paper_1307_6703_amd import Lattice
    T, lam, A0 = 0.95, 32, 1e-4
    N, Q = ls.table1_nq(T)
    U = GDOT * LY / 2
    fext = ls.sine_force(Lx, A0, lam)
    n0 = _zebra_n0(Lx, 7000 + Lx)
    _say("zebra configuration vs oracle", Lx, fp32)
    g = Lattice(Lx, LY, T=T, tau=1.0, kappa=0.3, N=N, Q=Q, U=U, fext=fext, fp32=fp32,
                check_every=100, drift_correct=bool(fp32))
    if fp32 is True:
        g.set_launch(128, 0, steps_per_launch=2)
    g.init(n0).step(100)
    n, ux, uy = g.moments()
    spl = g.steps_per_launch()
    g.close()
    if Lx not in _ZEBRA_ORACLE:
        o = OracleLB(Params(Lx, LY, T=T, tau=1.0, kappa=0.3, N=N, Q=Q, U=U), n0, fext=fext)
        o.run(100)
        _ZEBRA_ORACLE[Lx] = o
    o = _ZEBRA_ORACLE[Lx]
    du = max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max())
    err = np.abs(n - o.n).max() if fp32 is False else (np.abs(n - o.n) / o.n).max()
    _say(f"{spl} step(s) per launch: density error {err:.2e}, |du| {du:.2e}")
    assert err <= tol and du <= tol


def test_table2_rows_as_printed():
    # Every row of Table 2, each as its own lattice, 3e5 steps from a flat
    # interface: the amplitude here beside the printed one. tau is read in
    # the paper's units (reading c2); the tau = 2 and 3 rows are also run with
    # tau read in units of the time step (tau_l = tau), the other reading.
    # Asserted are the relations that hold: at T = 0.95 the amplitude does not
    # depend on lambda (the paper prints the same values for 32 and 64) nor on
    # A0, and it grows from Lx = 512 to 1024 at both temperatures. The
    # absolute amplitudes, the wave at Lx = 256, the lambda independence at
    # T = 0.91 and the tau dependence do not agree (parity unpinned; the
    # comparison is printed).
    import math
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1307_6703_amd import Batch
    rows = _table2()
    runs = []
    for r in rows:
        T, lam, tau, g, A0, kap, Lx, Ly, A = r
        runs.append((r, tau, "paper"))
        if tau != 1:
            runs.append((r, tau / math.sqrt(3.0), "dt"))
    specs, n0s = [], []
    for k, (r, tau_arg, _) in enumerate(runs):
        T, lam, tau, g, A0, kap, Lx, Ly, A = r
        N, Q = ls.table1_nq(T)
        nL, nV, _ = cf.maxwell(T)
        y = np.arange(Ly, dtype=np.float64)[:, None]
        prof = nV + (nL - nV) * 0.5 * (1.0 - np.tanh((y - Ly / 2) / 2.0))
        specs.append(dict(Lx=Lx, Ly=Ly, T=T, tau=tau_arg, kappa=kap, N=N, Q=Q, U=g * Ly / 2,
                          fext=ls.sine_force(Lx, A0, lam)))
        n0s.append(np.repeat(prof, Lx, axis=1) + (ls.noisy_density(Lx, Ly, 3000 + k) - 1.0))
    b = Batch(specs, fp32=True, check_every=1000, drift_correct=True)
    for i, n0 in enumerate(n0s):
        b.init(i, n0)
    b.autotune(nsteps=4)
    done, samples = 0, {i: [] for i in range(len(runs))}
    while done < STEPS:
        b.step(EVERY)
        b.drop_unstable()
        done += EVERY
        if done >= STEPS - 3 * EVERY:
            st = b.status()
            for i in range(len(runs)):
                if st[i] == 0:
                    samples[i].append(_amplitude(b.moments(i)[0], runs[i][0][0]))
        _say(f"step {done}")
    st = b.status()
    b.close()
    A = {}
    print("\nT     lam tau  A0     kappa Lx    tau read  A/Ly here  single-crossing  A/Ly paper")
    for i, (r, _, reading) in enumerate(runs):
        T, lam, tau, g, A0, kap, Lx, Ly, Ap = r
        if st[i] != 0:
            print(f"{T:.2f}  {lam:3d} {tau:.0f}   {A0:.0e}  {kap:.1f}   {Lx:5d} {reading:8s}  unstable"
                  f"         -                {Ap}")
            continue
        amps = [a for a, f in samples[i]]
        fr = min(f for _, f in samples[i])
        A[(T, lam, tau, A0, kap, Lx, reading)] = (float(np.mean(amps)), fr)
        print(f"{T:.2f}  {lam:3d} {tau:.0f}   {A0:.0e}  {kap:.1f}   {Lx:5d} {reading:8s}  "
              f"{np.mean(amps):.3f}      {fr:.2f}             {Ap}")
    for T in (0.95, 0.91):
        for Lx in (512, 1024):
            a32, f32 = A[(T, 32, 1.0, 1e-4, 0.3, Lx, "paper")]
            a64, f64 = A[(T, 64, 1.0, 1e-4, 0.3, Lx, "paper")]
            assert f32 == 1.0 and f64 == 1.0
            if T == 0.95:
                assert abs(a32 - a64) <= 0.03, (T, Lx, a32, a64)
        assert A[(T, 32, 1.0, 1e-4, 0.3, 1024, "paper")][0] >= \
            A[(T, 32, 1.0, 1e-4, 0.3, 512, "paper")][0] + 0.03
    for Lx in (512, 1024):
        assert abs(A[(0.95, 32, 1.0, 1e-4, 0.3, Lx, "paper")][0] -
                   A[(0.95, 32, 1.0, 1e-5, 0.3, Lx, "paper")][0]) <= 0.03
