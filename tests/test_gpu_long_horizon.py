"""FP32 storage against FP64 over long runs: the sixteen 1024 x 256 workloads
(T in {0.90, 0.95}, wall speed U in {0.005, 0.05}, four seeds), 50k steps,
the maximum relative density error every 1000 steps.

The reference is the FP64 path of the same library. It is a proxy for the
FP64 oracle, which is too slow for 50k steps at this size: the FP64 path
matches the oracle within 1e-13 on the 2000-step sheared parity workload and
within 1e-10 on every other parity case (tests/test_gpu_parity.py), 12 orders
below the 1e-4 gate checked here.

Two FP64 runs from perturbed n0 (one FP64 ulp, one FP32 ulp) show how the
scheme treats a single perturbation: it decays on these workloads, so the
gate is judged where the intrinsic floor lies far below it.

FP32 storage with FP64 arithmetic and stochastic rounding of the stored
values ("sr") holds 1e-4 on all sixteen workloads. FP32 arithmetic with
rounding to nearest makes the same rounding error at every node of a
uniform phase, step after step; the lattice integrates that bias over the
slow relaxation of momentum and of the phase pattern, and the error
settles at 2e-4 to 1e-3 on twelve workloads. Those are marked as expected
failures with the measured error; the other four are asserted."""
import sys

import numpy as np
import pytest

import lbsynth as ls

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CHECK = 1000
TOL = 1e-4
WORKS = ls.FP32_VS_FP64
NAMES = [w.name for w in WORKS]

# FP32 arithmetic, measured maximum over 50k steps (the same on every run:
# the path is deterministic)
FP32_MEASURED = {
    "T0.9-U0.005": "5.7e-4 to 9.6e-4",
    "T0.9-U0.05": "8.9e-4 to 1.02e-3",
    "T0.95-U0.05": "4.2e-4",
}


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def _run(torch, prec, drift, n0s, steps, ref=None):
    """Batch of all workloads. Without ref: density snapshots [checks, B, Ly, Lx];
    with ref: max relative density error against it [checks, B]. Also the
    relative mass drift per workload."""
    from paper_1307_6703_amd import Batch
    specs = [dict(Lx=w.Lx, Ly=w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                  fext=w.fext()) for w in WORKS]
    b = Batch(specs, fp32=prec, check_every=100 if prec else CHECK, drift_correct=drift)
    for i, n0 in enumerate(n0s):
        b.init(i, n0)
    m0 = np.array([b.reduce(i)["mass"] for i in range(len(WORKS))])
    out = []
    for j in range(steps // CHECK):
        b.step(CHECK)
        n = b.moments_device()[:, 0].cpu().numpy()
        out.append(n if ref is None else np.max(np.abs(n - ref[j]) / ref[j], axis=(1, 2)))
    m1 = np.array([b.reduce(i)["mass"] for i in range(len(WORKS))])
    status = b.status()
    b.close()
    assert all(s == 0 for s in status), status
    return np.stack(out), np.abs(m1 - m0) / m0


@pytest.fixture(scope="module")
def runs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    steps = WORKS[0].steps
    n0s = [w.n0() for w in WORKS]
    # one FP64 ulp up everywhere (the scheme's amplification of rounding), and
    # one FP32 ulp up (perturbations of the size FP32 storage makes)
    n0p = [np.nextafter(n, 2.0) for n in n0s]
    n0q = [n.astype(np.float32).astype(np.float64) + np.spacing(n.astype(np.float32)).astype(np.float64)
           for n in n0s]
    r = {}
    _say("fp64 reference")
    ref, r["dm64"] = _run(torch, 0, False, n0s, steps)
    _say("fp64 one fp64 ulp off")
    r["floor64"], _ = _run(torch, 0, False, n0p, steps, ref)
    _say("fp64 one fp32 ulp off")
    r["floor32"], _ = _run(torch, 0, False, n0q, steps, ref)
    _say("fp32 storage, fp64 arithmetic, stochastic rounding, drift correction")
    r["sr"], r["dm_sr"] = _run(torch, "sr", True, n0s, steps, ref)
    _say("fp32 with drift correction")
    r["fp32"], r["dm32"] = _run(torch, True, True, n0s, steps, ref)
    _say("fp32 without drift correction")
    r["fp32n"], r["dm32n"] = _run(torch, True, False, n0s, steps, ref)
    t = (np.arange(len(ref)) + 1) * CHECK
    print("\nmax relative density error vs FP64 over the 16 workloads, and the two floors")
    print(" step    sr         fp32+corr   fp32        floor(64-ulp) floor(32-ulp)")
    for j in [0, 1, 4, 9, 19, 29, 39, 49]:
        if j < len(t):
            print(f"{t[j]:6d}  {r['sr'][j].max():9.2e}  {r['fp32'][j].max():9.2e}  "
                  f"{r['fp32n'][j].max():9.2e}  {r['floor64'][j].max():9.2e}     "
                  f"{r['floor32'][j].max():9.2e}")
    print("per workload, max over the run: sr, fp32 (floors at 50k)")
    for i, w in enumerate(WORKS):
        print(f"  {w.name}: sr {r['sr'][:, i].max():.2e}, fp32 {r['fp32'][:, i].max():.2e} "
              f"(floors {r['floor64'][-1, i]:.2e} / {r['floor32'][-1, i]:.2e})")
    print(f"mass drift: fp64 max {r['dm64'].max():.2e}, sr+corr max {r['dm_sr'].max():.2e}, "
          f"fp32+corr max {r['dm32'].max():.2e}, fp32 max {r['dm32n'].max():.2e}", flush=True)
    return r


@pytest.mark.parametrize("i", range(len(WORKS)), ids=NAMES)
def test_sr_storage_within_1e4_of_fp64(runs, i):
    assert runs["sr"][:, i].max() <= TOL, (NAMES[i], runs["sr"][:, i].max())


def _fp32_case(i):
    w = WORKS[i]
    key = f"T{w.T}-U{w.U}"
    if key in FP32_MEASURED:
        return pytest.param(i, id=NAMES[i], marks=pytest.mark.xfail(
            strict=True, reason=f"FP32 arithmetic settles at {FP32_MEASURED[key]} on {key} "
                                f"(a rounding bias integrated by slow modes)"))
    return pytest.param(i, id=NAMES[i])


@pytest.mark.parametrize("i", [_fp32_case(i) for i in range(len(WORKS))])
def test_fp32_arithmetic_within_1e4_of_fp64(runs, i):
    assert runs["fp32"][:, i].max() <= TOL, (NAMES[i], runs["fp32"][:, i].max())


def test_fp32_arithmetic_error_settles(runs):
    # the FP32-arithmetic error reaches a level and stays there: no secular growth
    e = runs["fp32"]
    for i in range(len(WORKS)):
        assert e[-10:, i].max() <= 2.0 * e[10:40, i].max() + 1e-5, NAMES[i]


def test_single_perturbations_decay_and_mass(runs):
    # a single perturbation decays: no chaotic amplification on these workloads
    assert runs["floor64"][-1].max() <= runs["floor64"][:5].max()
    assert runs["floor32"][-1].max() <= 1e-4
    assert runs["dm64"].max() <= 5e-12
    assert runs["dm32"].max() <= 1e-6
    assert runs["dm_sr"].max() <= 1e-6
