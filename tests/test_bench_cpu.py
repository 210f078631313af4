"""Host-side parts of the benchmark: the one-GPU guard and the CPU baseline
leg (the FP64 oracle on a small matrix)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_cpu_baseline_leg_times_the_oracle():
    sys.path.insert(0, ROOT)
    import bench
    A = np.random.Generator(np.random.PCG64(5)).standard_normal((96, 96))
    per_rep, cores, reps = bench.cpu_baseline(A, 16, 4, 7, budget_s=0.05)
    assert per_rep > 0 and cores >= 1 and 1 <= reps <= 50


def test_traffic_figure_needs_matching_sources(tmp_path, monkeypatch):
    """The recorded HBM traffic is reported only for the kernel sources it was
    measured on."""
    sys.path.insert(0, ROOT)
    import bench
    f = tmp_path / "traffic.txt"
    f.write_text("source_digest: %s\nhbm_bytes_per_launch: 123.0\n" % bench.sources_digest())
    assert bench.recorded_traffic(str(f)) == 123.0
    f.write_text("source_digest: 0000000000000000\nhbm_bytes_per_launch: 123.0\n")
    assert bench.recorded_traffic(str(f)) is None
    assert bench.recorded_traffic(str(tmp_path / "missing.txt")) is None


def test_cpu_baseline_extras():
    """One-thread timing and the oracle's adaptive HSS run on the n = 1024
    kernel workload, which stops at d = 64 at its tolerance."""
    sys.path.insert(0, ROOT)
    import bench
    A = np.random.Generator(np.random.PCG64(6)).standard_normal((128, 128))
    ex = bench.cpu_baseline_extras(A, 16, 4, 7)
    assert ex["one_thread"]["s_per_step"] > 0
    h = ex["hss_1024_compress"]
    assert h["converged"] and h["final_d"] == 64 and h["s"] > 0
