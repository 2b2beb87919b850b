"""FP32 deviation storage against FP64 over long runs (1024x256, 50k steps).

The FP64 GPU path is pinned to the oracle at 1e-10, so it serves as the
reference. Two FP64 runs from perturbed n0 (one FP64 ulp, one FP32 ulp) show
how the scheme treats a single perturbation: it decays here (the floors fall
over time). FP32 arithmetic instead injects about 1e-7 every step, and a
steady state shifts by that amount times the relaxation time of its slowest
modes (thousands of steps for stripes of 128-256 nodes; longer where phase
interfaces can move almost freely). So FP32 stays within 1e-4 of FP64 only
on the weakly driven T = 0.95 workloads; on the others the error settles at
4e-4 to 1e-3 and does not grow. The test asserts exactly that, and the mass
drift with the FP32 drift correction."""
import sys

import numpy as np
import pytest

import lbsynth as ls

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

CHECK = 1000


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _run(torch, works, fp32, drift, n0s, steps, ref=None):
    """Batch of all workloads. Without ref: density snapshots [checks, B, Ly, Lx];
    with ref: max relative density error against it [checks, B]. Also the
    relative mass drift per workload."""
    from paper_1307_6703_amd import Batch
    specs = [dict(Lx=w.Lx, Ly=w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                  fext=w.fext()) for w in works]
    b = Batch(specs, fp32=fp32, check_every=100 if fp32 else CHECK, drift_correct=drift)
    for i, n0 in enumerate(n0s):
        b.init(i, n0)
    m0 = np.array([b.reduce(i)["mass"] for i in range(len(works))])
    out = []
    for j in range(steps // CHECK):
        b.step(CHECK)
        n = b.moments_device()[:, 0].cpu().numpy()
        out.append(n if ref is None else np.max(np.abs(n - ref[j]) / ref[j], axis=(1, 2)))
    m1 = np.array([b.reduce(i)["mass"] for i in range(len(works))])
    status = b.status()
    b.close()
    assert all(s == 0 for s in status), status
    return np.stack(out), np.abs(m1 - m0) / m0


def test_fp32_against_fp64_long_horizon(torch_cuda):
    torch = torch_cuda
    works = ls.FP32_VS_FP64
    steps = works[0].steps
    n0s = [w.n0() for w in works]
    # one FP64 ulp up everywhere (the scheme's amplification of rounding), and
    # one FP32 ulp up (perturbations of the size FP32 storage makes)
    n0p = [np.nextafter(n, 2.0) for n in n0s]
    n0q = [n.astype(np.float32).astype(np.float64) + np.spacing(n.astype(np.float32)).astype(np.float64)
           for n in n0s]
    _say("fp64 reference")
    ref, dm64 = _run(torch, works, False, False, n0s, steps)
    _say("fp64 one fp64 ulp off")
    floor64, _ = _run(torch, works, False, False, n0p, steps, ref)
    _say("fp64 one fp32 ulp off")
    floor32, _ = _run(torch, works, False, False, n0q, steps, ref)
    _say("fp32 with drift correction")
    e32, dm32 = _run(torch, works, True, True, n0s, steps, ref)
    _say("fp32 without drift correction")
    e32n, dm32n = _run(torch, works, True, False, n0s, steps, ref)
    t = (np.arange(len(ref)) + 1) * CHECK
    print("\nmax relative density error vs FP64 over the 16 workloads, and the two floors")
    print(" step    fp32+corr   fp32        floor(64-ulp) floor(32-ulp)")
    for j in [0, 1, 4, 9, 19, 29, 39, 49]:
        if j < len(t):
            print(f"{t[j]:6d}  {e32[j].max():9.2e}  {e32n[j].max():9.2e}  {floor64[j].max():9.2e}"
                  f"     {floor32[j].max():9.2e}")
    print("per workload: fp32 max error over the run, last 10k steps, and at 50k")
    for i, w in enumerate(works):
        print(f"  {w.name}: max {e32[:, i].max():.2e}, last 10k {e32[-10:, i].max():.2e}, "
              f"50k {e32[-1, i]:.2e} (floors {floor64[-1, i]:.2e} / {floor32[-1, i]:.2e})")
    print(f"mass drift: fp64 max {dm64.max():.2e}, fp32+corr max {dm32.max():.2e}, "
          f"fp32 max {dm32n.max():.2e}")
    for i, w in enumerate(works):
        # a settled error, no secular growth
        assert e32[-10:, i].max() <= 2.0 * e32[10:40, i].max() + 1e-5, w.name
        assert e32[:, i].max() <= 2e-3, w.name
        if w.T >= 0.95 and w.U <= 0.005:
            assert e32[:, i].max() <= 1e-4, w.name
    # single perturbations decay: no chaotic amplification on these workloads
    assert floor64[-1].max() <= floor64[:5].max()
    assert dm64.max() <= 5e-12
    assert dm32.max() <= 1e-6
