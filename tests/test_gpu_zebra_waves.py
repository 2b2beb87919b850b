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
