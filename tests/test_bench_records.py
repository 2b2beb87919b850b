"""bench.py's committed measurement records stay attached to the code they
measured (CPU only)."""
import json
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_traffic_record_matches_the_step_kernel_source():
    # the HBM traffic from rocprofv3 counters is reported only while the
    # step kernels' source hash matches the one recorded with the counters
    t = json.load(open(bench.TRAFFIC_FILE))
    assert t["kernel_source_sha256"] == bench.kernel_hash(), \
        "the step kernels changed since the counters were taken: take them again"
    assert bench.measured_traffic(t["nodes"], t["steps_per_launch"], *t["launch"]) == \
        t["traffic_bytes_per_launch"]
    # and only for the launch shape they were taken on
    assert bench.measured_traffic(t["nodes"], t["steps_per_launch"], t["launch"][0],
                                  t["launch"][1] + 8) is None
    # the counters see about the algorithmic bytes or more, never far less
    assert 0.5 * t["algorithmic_bytes_per_launch"] / t["steps_per_launch"] <= \
        t["traffic_bytes_per_launch"] <= 2 * t["algorithmic_bytes_per_launch"]


def test_kernel_hash_ignores_comments_and_other_kernels(tmp_path, monkeypatch):
    src = open(bench.KERNEL_SOURCE).read()
    cut = src.index(bench.KERNEL_SECTION_END)
    h0 = bench.kernel_hash()
    edited = src[:cut] + "// a comment\n" + src[cut:] + "\nint unrelated_kernel_code;\n"
    p = tmp_path / "k.hip"
    p.write_text(edited)
    monkeypatch.setattr(bench, "KERNEL_SOURCE", str(p))
    assert bench.kernel_hash() == h0
    p.write_text(src[:cut].replace("const int u = t + 1;", "const int u = t + 2;") + src[cut:])
    assert bench.kernel_hash() != h0


def test_bench_refuses_more_than_one_gpu():
    # one GPU's throughput only: --gpus N > 1 exits with a message, before any
    # device work
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one MI355X" in r.stderr


def test_d2q17_workload_is_the_headline_lattice_periodic():
    import lbsynth as ls
    w, h = ls.D2Q17_WORKLOAD, ls.ROOFLINE
    assert (w.Lx, w.Ly, w.T, w.V0, w.k, w.seed) == (h.Lx, h.Ly, h.T, h.V0, h.k, h.seed)
    assert w.y_periodic and w.U == 0.0
    assert bench.BYTES_PER_UPDATE_D2Q17_FP32 == 2 * 17 * 4
