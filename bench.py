#!/usr/bin/env python3
"""Throughput of the fused lattice Boltzmann step on one MI355X.

Workload (synthetic, seeded): 8192 x 2048 lattice between walls moving at
+-0.08, T = 0.9 T_c, periodic potential V0 = 0.01 with 32 stripes, density noise
+-0.01 around n = 1, FP32 deviation storage, FP64 mass/momentum check with
drift correction every 100 steps. One step = one full time step of the lattice
(stream, density, stencils, force, walls, collision, store) plus its share of
the checks.

Order of the measurements: the step kernel alone (checks off) for the
roofline, then, queued behind it on the same lattice with no idle gap, the
--warmup and --steps of the headline with the checks; then the cost of a
check, the other precisions on the same lattice, the D2Q17 variant on its
periodic workload of the same size, the batched sweep, the learned surrogate
and the CPU oracle.

The default launch runs two steps per launch (the two-step kernel keeps the
first step's populations on chip). The roofline counts 72 algorithmic bytes
per node update (nine populations read and written in FP32), times the
updates of one launch, over the launch's duration; with two steps per launch
the populations cross HBM once per two updates, so that figure is an
effective rate, hbm_gbs_min the rate of the bytes that must cross HBM and
hbm_gbs_measured that of the bytes the HBM counters saw.

Prints one JSON line: MLUPS (million lattice-node updates per second), the
roofline of the step kernel against the HBM peak, the FP64 CPU oracle timed
on the host cores on a bounded sample of the same workload, and the headline
path's difference from the oracle after the sample's steps from the same
fields (error_vs_oracle).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
BYTES_PER_UPDATE_FP32 = 72     # 9 populations read + 9 written, 4 B each
BYTES_PER_UPDATE_FP64 = 144
BYTES_PER_UPDATE_D2Q17_FP32 = 136   # 17 populations read + 17 written, 4 B each
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernel_traffic.json")
KERNEL_SOURCE = os.path.join(ROOT, "paper_1307_6703_amd", "csrc", "lb_device.hip")
TUNED = os.path.join(ROOT, "paper_1307_6703_amd", "tuned_launch.json")


# The two-step kernel and everything it compiles from come first in
# KERNEL_SOURCE; the one-step kernel, the initial-state, check and conversion
# kernels follow this line.
KERNEL_SECTION_END = "// ---- one-step kernel"


def kernel_hash() -> str:
    """SHA-256 prefix of the two-step kernel's source (KERNEL_SOURCE up to
    KERNEL_SECTION_END) with comments and blank space removed, so that
    counters stay attached to the code they measured."""
    import re
    src = open(KERNEL_SOURCE).read()
    cut = src.find(KERNEL_SECTION_END)
    if cut >= 0:
        src = src[:cut]
    src = re.sub(r"//[^\n]*", "", src)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()[:16]


def tuned_launch(key: str):
    try:
        return json.load(open(TUNED)).get(key)
    except (OSError, ValueError):
        return None


def measured_traffic(nodes: int, steps_per_launch: int, threads: int, rows: int):
    """HBM bytes per launch from committed rocprofv3 counters, if they were
    taken on the current kernel source for the kernel and launch shape that
    run."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if (t.get("kernel_source_sha256") != kernel_hash() or t.get("nodes") != nodes
            or t.get("steps_per_launch", 1) != steps_per_launch
            or t.get("launch") != [threads, rows]):
        return None
    return t.get("traffic_bytes_per_launch")


def cpu_baseline(w, n0, fext, seconds: float):
    """The FP64 oracle as it stands, on the full lattice, for as many whole
    steps as fit in about `seconds` (at least one): on all host threads, then
    on one thread for about a third of that."""
    from oracle.lb_oracle import OracleLB, Params

    def timed(threads, budget):
        o = OracleLB(Params(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                            y_periodic=w.y_periodic), n0, fext=fext)
        t0 = time.perf_counter()
        used = o.run(1, threads=threads)
        t1 = time.perf_counter()
        steps = max(0, int(budget / max(t1 - t0, 1e-9)) - 1)
        if steps:
            o.run(steps, threads=threads)
        dt = time.perf_counter() - t0
        return round(w.nodes * (steps + 1) / dt / 1e6, 3), used, steps + 1, dt, o

    v, used, n, dt, o = timed(0, seconds)
    v1, _, n1, dt1, _ = timed(1, seconds / 3)
    return {"value": v, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"{n} FP64 steps of the full {w.Lx}x{w.Ly} lattice ({dt:.1f} s)",
            "single_thread": {"value": v1, "unit": "MLUPS", "cores": 1,
                              "sample": f"{n1} FP64 steps of the full lattice on one thread "
                                        f"({dt1:.1f} s)"}}, o, n


def error_vs_oracle(w, n0, fext, o, steps: int, check_every: int):
    """The headline path (FP32 deviations, its default launch) run for the
    same steps from the same fields as the oracle's all-thread sample: the
    largest relative density and absolute velocity differences over the
    lattice."""
    import numpy as np
    from paper_1307_6703_amd import Lattice
    lat = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                  y_periodic=w.y_periodic, fp32=True, check_every=check_every, drift_correct=True)
    lat.init(n0)
    lat.step(steps)
    n, ux, uy = lat.moments()
    launch = lat.get_launch()
    spl = lat.steps_per_launch()
    lat.close()
    return {"steps": steps, "max_rel_density": float(np.max(np.abs(n - o.n) / o.n)),
            "max_abs_velocity": float(max(np.abs(ux - o.ux).max(), np.abs(uy - o.uy).max())),
            "tolerance": 1e-4, "path": f"fp32, launch {launch[0]} x {launch[1]}, {spl} step(s) per launch"}


def batched_bench(steps: int, seed: int = 1307, launch=None):
    """The batched sweep: 96 uneven lattices advanced together (one launch per
    step over all their tiles, HIP-graph replay), autotuned launch shape
    unless `launch` = (threads, rows, steps per launch) fixes it.
    Returns aggregate MLUPS = sum of nodes x steps / time."""
    import torch
    import lbsynth as ls
    from paper_1307_6703_amd import Batch
    def batch_of(draws):
        specs = [dict(Lx=w.Lx, Ly=w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U,
                      fext=w.fext()) for w in draws]
        b = Batch(specs, fp32=True, check_every=100, drift_correct=True)
        for i, w in enumerate(draws):
            b.init(i, w.n0())
        return b

    # a draw whose lattice fails a stability check within the run (a deep
    # quench under strong shear can) is replaced by the next draw; the
    # screening covers the autotuner's steps (about 4000), the warm-up and the
    # timed steps
    pool = ls.batch_draws(128, seed=seed)
    scr = batch_of(pool)
    scr.step(steps + 5000)
    status = scr.status()
    scr.close()
    draws = [w for w, st in zip(pool, status) if st == 0][:96]
    replaced = pool.index(draws[-1]) + 1 - len(draws)
    b = batch_of(draws)
    if launch is None:
        # 100 timed steps per candidate: every candidate's window holds
        # exactly one of the checks (every 100 steps), so none is favoured
        th, rw, _ = b.autotune(nsteps=100)
    else:
        th, rw = launch[0], launch[1]
        b.set_launch(th, rw, steps_per_launch=launch[2] if len(launch) > 2 else 1)
    b.step(100)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    status = b.status()
    out = {"instances": len(draws), "nodes": b.nodes, "steps": steps,
           "MLUPS": round(b.nodes * steps / (ms * 1e-3) / 1e6, 1),
           "ms_per_step": round(ms / steps, 4),
           "launch": {"threads": th, "rows": rw, "steps_per_launch": b.steps_per_launch()},
           "unstable_instances": sum(1 for v in status if v != 0),
           "draws_replaced_unstable": replaced,
           # 72 algorithmic bytes per node update; the two population buffers
           # (2 x 36 B per node) exceed the 256 MB Infinity Cache, so the batch
           # streams from HBM rather than running cache-resident
           "algorithmic_gbs": round(BYTES_PER_UPDATE_FP32 * b.nodes * steps / (ms * 1e-3) / 1e9, 1),
           "algorithmic_frac_of_peak": round(BYTES_PER_UPDATE_FP32 * b.nodes * steps /
                                             (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
           "population_buffers_mb": round(2 * 36 * b.nodes / 1e6, 1),
           "cache_resident": 2 * 36 * b.nodes < 256e6,
           "workload": "96 draws: Lx in {128..1024}, Ly in {64,128,256}, T in [0.85,0.98], "
                       "V0 in [0,0.02], k in {2,4,8}, U in [0,0.08], FP32"}
    b.close()
    return out


def mode_bench(w, n0_dev, fext, prec: int, steps: int, check_every: int):
    """Throughput of another precision on the headline lattice in its default
    launch: `steps` timed steps with the FP64 checks, after 20 warm-up steps;
    the step kernel's roofline at 72 (FP32 storage) or 144 (FP64) algorithmic
    bytes per node update."""
    import torch
    from paper_1307_6703_amd import Lattice
    lat = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                  y_periodic=w.y_periodic, fp32=prec, check_every=check_every, drift_correct=prec != 0)
    lat.init(n0_dev)
    threads, rows, blocks = lat.get_launch()
    lat.step(20)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    lat.step(steps)
    ev[1].record()
    lat.set_checks(0, False)
    ev[2].record()
    lat.step(steps)
    ev[3].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[1]) / steps
    k_ms = ev[2].elapsed_time(ev[3]) / steps
    bpu = BYTES_PER_UPDATE_FP64 if prec == 0 else BYTES_PER_UPDATE_FP32
    red = lat.reduce()
    lat.close()
    achieved = bpu * w.nodes / (k_ms * 1e-3) / 1e9
    return {"MLUPS": round(w.nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
            "steps": steps,
            "launch": {"threads": threads, "rows": rows, "workgroups": blocks, "steps_per_launch": 1},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "kernel": ("step_kernel<float, double, %d, false, false>" if prec == 2 else
                                    "step_kernel<double, double, %d, false, false>") % threads,
                         "us_per_launch": round(k_ms * 1e3, 2), "bytes_per_update": bpu},
            "nmin": red["nmin"], "nmax": red["nmax"]}


def d2q17_bench(steps: int, check_every: int):
    """The D2Q17 variant (the third-order model named after Eq.(nav)) on its
    workload, 8192 x 2048 periodic, FP32 storage, in its default launch:
    `steps` timed steps with the FP64 checks and drift correction after 20
    warm-up steps, then the same number without checks for the step kernel's
    roofline at 136 algorithmic bytes per node update."""
    import torch
    import lbsynth as ls
    from paper_1307_6703_amd import Lattice17
    w = ls.D2Q17_WORKLOAD
    lat = Lattice17(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, fext=w.fext(),
                    fp32=True, check_every=check_every, drift_correct=True)
    lat.init(w.n0())
    threads, rows, blocks = lat.get_launch()
    m0 = lat.reduce()["mass"]
    lat.step(20)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    lat.step(steps)
    ev[1].record()
    torch.cuda.synchronize()
    red = lat.reduce()
    lat.close()
    # the kernel alone: a lattice without checks, queued steps
    k = Lattice17(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, fext=w.fext(),
                  fp32=True)
    k.init(w.n0())
    k.step(20)
    ev[2].record()
    k.step(steps)
    ev[3].record()
    torch.cuda.synchronize()
    k.close()
    # FP32 storage with FP64 arithmetic and stochastic rounding, kernel alone
    sr = Lattice17(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, fext=w.fext(),
                   fp32="sr")
    sr.init(w.n0())
    sr_launch = sr.get_launch()
    sr.step(20)
    e4, e5 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e4.record()
    sr.step(steps)
    e5.record()
    torch.cuda.synchronize()
    sr.close()
    ms = ev[0].elapsed_time(ev[1]) / steps
    k_ms = ev[2].elapsed_time(ev[3]) / steps
    sr_ms = e4.elapsed_time(e5) / steps
    bpu = BYTES_PER_UPDATE_D2Q17_FP32
    achieved = bpu * w.nodes / (k_ms * 1e-3) / 1e9
    assert red["nonfinite"] == 0 and 0 < red["nmin"] and red["nmax"] < 3, red
    return {"workload": w.name, "Lx": w.Lx, "Ly": w.Ly, "T": w.T, "V0": w.V0, "stripes": w.k,
            "MLUPS": round(w.nodes / (ms * 1e-3) / 1e6, 1), "ms_per_step": round(ms, 5),
            "steps": steps, "checks": f"fp64 every {check_every} steps + drift correction",
            "launch": {"threads": threads, "rows": rows, "workgroups": blocks,
                       "steps_per_launch": 1},
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "kernel": "step17_kernel<float, float, %d, false>" % threads,
                         "us_per_launch": round(k_ms * 1e3, 2), "bytes_per_update": bpu},
            "mass_drift": abs(red["mass"] - m0) / m0, "nmin": red["nmin"], "nmax": red["nmax"],
            "fp32_storage_fp64_arithmetic_sr": {
                "MLUPS_kernel": round(w.nodes / (sr_ms * 1e-3) / 1e6, 1),
                "us_per_launch": round(sr_ms * 1e3, 2),
                "achieved_gbs": round(bpu * w.nodes / (sr_ms * 1e-3) / 1e9, 1),
                "launch": {"threads": sr_launch[0], "rows": sr_launch[1],
                           "workgroups": sr_launch[2]}}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000,
                    help="timed steps of the headline lattice (10k, about 1.7 s)")
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--launch", default=None,
                    help="threads,rows[,steps per launch] of the step kernel (steps 2: the "
                         "two-step kernel)")
    ap.add_argument("--autotune", action="store_true", help="autotune the launch shape first")
    ap.add_argument("--check-every", type=int, default=100)
    ap.add_argument("--roofline-steps", type=int, default=2000,
                    help="steps of the step kernel alone (checks off) timed for the roofline, "
                         "before the headline's warm-up and timed steps")
    ap.add_argument("--mode-steps", type=int, default=400,
                    help="timed steps of the FP32-storage FP64-arithmetic mode and of FP64 on the "
                         "headline lattice (0: skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--batched-steps", type=int, default=20000,
                    help="timed steps of the 96-lattice batched sweep reported beside the "
                         "headline (20k, about 2.3 s; 0: skip)")
    ap.add_argument("--batched-launch", default=None,
                    help="threads,rows[,steps per launch] of the batched sweep (default: autotuned)")
    ap.add_argument("--surrogate-seconds", type=float, default=30.0,
                    help="training time limit of the learned surrogate reported beside the "
                         "headline (0: skip)")
    ap.add_argument("--surrogate-iters", type=int, default=20000,
                    help="Adam steps of the surrogate's training; the learning-rate schedule "
                         "runs over them unless the time limit ends it first (then the result "
                         "depends on the device's speed)")
    ap.add_argument("--d2q17-steps", type=int, default=400,
                    help="timed steps of the D2Q17 variant on its workload (0 skips it)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of 1 GiB (for scaling HBM counters)")
    args = ap.parse_args()

    if args.copy_calibration:
        import torch
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": src.numel() * 4, "copy_bytes_written": dst.numel() * 4,
                          "launches": 3}), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one MI355X: the lattice fits one GPU's HBM and this library "
              "has no multi-GPU path; run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import lbsynth as ls
    from paper_1307_6703_amd import Lattice

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    w = ls.ROOFLINE
    n0, fext = w.n0(), w.fext()
    n0_dev = torch.from_numpy(n0).cuda()
    lat = Lattice(w.Lx, w.Ly, T=w.T, tau=w.tau, kappa=w.kappa, N=w.N, Q=w.Q, U=w.U, fext=fext,
                  y_periodic=w.y_periodic, fp32=True, check_every=args.check_every,
                  drift_correct=True)
    lat.init(n0_dev)
    key = f"{w.Lx}x{w.Ly}-fp32-gfx950"
    if args.launch:
        lat.set_launch(*(int(v) for v in args.launch.split(",")))
    elif args.autotune:
        lat.autotune(nsteps=10)
    elif tuned_launch(key):
        lat.set_launch(*tuned_launch(key))
    threads, rows, blocks = lat.get_launch()
    spl = lat.steps_per_launch()
    print(f"[bench] {w.name}: {w.nodes} nodes, launch {threads} threads x {rows} rows, "
          f"{blocks} workgroups, {spl} step(s) per launch", file=sys.stderr, flush=True)

    m0 = lat.reduce()["mass"]
    # 1. the step kernel alone (checks off), for the roofline: a whole number of
    # launches after 200 warm-up launches.
    lat.set_checks(0, False)
    lat.step(200 * spl)
    k_steps = max(spl, args.roofline_steps // spl * spl)
    e2, e3 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e2.record()
    lat.step(k_steps)
    e3.record()

    # 2. the headline: the same lattice, W warm-up steps, then exactly K timed
    # steps with the FP64 checks and drift correction. They are queued behind
    # the roofline's steps with no host synchronisation in between: a device
    # that has idled for tens of milliseconds runs its next few launches at
    # lower clocks (a 20-step window after a 50 ms idle measured 4.4 ms
    # against 3.6 ms queued behind work), which a window of a few launches
    # would measure instead of the step.
    lat.set_checks(args.check_every, True)
    base = lat.step_count
    lat.step(args.warmup)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    lat.step(args.steps)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    k_ms = e2.elapsed_time(e3) / (k_steps // spl)  # per launch
    # algorithmic bytes: 72 B per node update, times the updates of a launch
    alg_bytes = BYTES_PER_UPDATE_FP32 * w.nodes * spl
    achieved = alg_bytes / (k_ms * 1e-3) / 1e9
    print(f"[bench] step kernel {k_ms * 1e3:.1f} us/launch ({spl} step(s)), {achieved:.0f} GB/s "
          f"algorithmic", file=sys.stderr, flush=True)
    ms = e0.elapsed_time(e1)
    mlups = w.nodes * args.steps / (ms * 1e-3) / 1e6
    ce = args.check_every
    s0 = base + args.warmup
    checks_in = 0 if ce <= 0 else (s0 + args.steps) // ce - s0 // ce
    print(f"[bench] timed {args.steps} steps (steps {s0 + 1} to {s0 + args.steps} of the run): "
          f"{ms:.1f} ms (wall {wall * 1e3:.1f} ms), {checks_in} check(s) among them",
          file=sys.stderr, flush=True)
    red = lat.reduce()

    # 3. what a check costs: 10 check intervals with and without the checks
    # (a check adds its FP64 reduction and makes the step before it a single
    # step); the headline's window holds checks_in of them
    chk = None
    if ce > 0:
        span = 10 * ce
        lat.step((-lat.step_count) % ce)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        lat.step(span)
        ev[1].record()
        lat.set_checks(0, False)
        ev[2].record()
        lat.step(span)
        ev[3].record()
        torch.cuda.synchronize()
        per = (ev[0].elapsed_time(ev[1]) - ev[2].elapsed_time(ev[3])) / 10
        due = args.steps / ce
        chk = {"every": ce, "in_timed_steps": checks_in, "ms_per_check": round(per, 4),
               "MLUPS_checks_amortised": round(
                   w.nodes * args.steps / ((ms + (due - checks_in) * per) * 1e-3) / 1e6, 1)}

    # the same bytes moved by a plain device copy: the streaming rate this
    # GPU reaches in practice (read + write), for context beside the peak
    src = torch.empty(w.nodes * 9, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e4, e5 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e4.record()
    for _ in range(10):
        dst.copy_(src)
    e5.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * src.numel() * 4 / (e4.elapsed_time(e5) / 10 * 1e-3) / 1e9
    del src, dst

    traffic = measured_traffic(w.nodes, spl, threads, rows)
    out = {
        "metric": "MLUPS",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "timed_steps_of_run": [s0 + 1, s0 + args.steps],
        "config": {"workload": w.name, "Lx": w.Lx, "Ly": w.Ly, "walls": not w.y_periodic,
                   "T": w.T, "tau": w.tau, "kappa": w.kappa, "N": w.N, "Q": w.Q, "U": w.U,
                   "V0": w.V0, "stripes": w.k, "seed": w.seed, "storage": "fp32-deviation",
                   "arithmetic": "fp32",
                   "checks": f"fp64 every {args.check_every} steps + drift correction",
                   "launch": {"threads": threads, "rows": rows, "workgroups": blocks,
                              "steps_per_launch": spl}},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # template arguments as the trace names them: strip threads, moments
                     # store, y boundary (1 walls, 2 periodic), regularised collision
                     "kernel": ("step2_kernel<%d, false, %d, false>" % (threads, 2 if w.y_periodic else 1)
                                if spl == 2 else "step_kernel<float, float, %d, false, false>" % threads),
                     "us_per_launch": round(k_ms * 1e3, 2),
                     "launches_timed": k_steps // spl,
                     "node_updates_per_launch": w.nodes * spl,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     # the bytes a launch must move through HBM: each population
                     # is read and written once per launch, whatever its steps
                     "hbm_bytes_per_launch_min": BYTES_PER_UPDATE_FP32 * w.nodes,
                     "hbm_gbs_min": round(BYTES_PER_UPDATE_FP32 * w.nodes / (k_ms * 1e-3) / 1e9, 1),
                     "hbm_gbs_measured": (round(traffic / (k_ms * 1e-3) / 1e9, 1)
                                          if traffic else None),
                     "hbm_frac_measured": (round(traffic / (k_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
                                           if traffic else None),
                     "note": ("two steps per launch: achieved counts 72 B per node update, times "
                              "the launch's two updates per node (the scope's algorithmic bytes), "
                              "an effective rate; the populations cross HBM once per launch "
                              "(hbm_gbs_min, hbm_gbs_measured); the launch takes as long as its "
                              "strips' memory access pattern, not HBM bandwidth or arithmetic" if spl == 2 else
                              "one step per launch: HBM-bound streaming of the populations"),
                     "copy_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "checks": chk,
        "hbm_frac_of_peak": round(mlups * 1e6 * BYTES_PER_UPDATE_FP32 / 1e9 / HBM_PEAK_GBS, 4),
        "mass_drift": abs(red["mass"] - m0) / m0,
        "gpu": torch.cuda.get_device_name(0),
    }
    assert red["nonfinite"] == 0 and 0 < red["nmin"] and red["nmax"] < 3, red
    lat.close()
    del lat
    torch.cuda.empty_cache()
    if args.mode_steps > 0:
        out["modes"] = {}
        for name, prec in (("fp32_storage_fp64_arithmetic_sr", 2), ("fp64", 0)):
            out["modes"][name] = mode_bench(w, n0_dev, fext, prec, args.mode_steps, args.check_every)
            print(f"[bench] {name}: {out['modes'][name]['MLUPS']} MLUPS, step kernel "
                  f"{out['modes'][name]['roofline']['us_per_launch']} us", file=sys.stderr, flush=True)
            torch.cuda.empty_cache()
    if args.d2q17_steps > 0:
        out["d2q17"] = d2q17_bench(args.d2q17_steps, args.check_every)
        print(f"[bench] d2q17: {out['d2q17']['MLUPS']} MLUPS, step kernel "
              f"{out['d2q17']['roofline']['us_per_launch']} us", file=sys.stderr, flush=True)
        torch.cuda.empty_cache()
    if args.batched_steps > 0:
        bl = tuple(int(v) for v in args.batched_launch.split(",")) if args.batched_launch else None
        out["batched"] = batched_bench(args.batched_steps, launch=bl)
        print(f"[bench] batched: {out['batched']['MLUPS']} MLUPS", file=sys.stderr, flush=True)
    if args.surrogate_seconds > 0:
        from paper_1307_6703_amd import surrogate
        out["surrogate"] = surrogate.experiment(
            train_seconds=args.surrogate_seconds, iters=args.surrogate_iters,
            log=lambda m: print(f"[bench] surrogate {m}", file=sys.stderr, flush=True))
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"], orc, orc_steps = cpu_baseline(w, n0, fext, args.cpu_seconds)
        out["error_vs_oracle"] = error_vs_oracle(w, n0, fext, orc, orc_steps, args.check_every)
        del orc
        print(f"[bench] against the FP64 oracle after {orc_steps} steps: max relative density "
              f"difference {out['error_vs_oracle']['max_rel_density']:.2e}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
