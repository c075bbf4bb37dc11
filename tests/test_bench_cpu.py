"""Host-side pieces of bench.py (no GPU): workloads carry the storage precision, the CPU baseline
runs the FP64 oracle on them, and more than one GPU is refused with a message."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_workloads_carry_precision_and_the_oracle_baseline_runs():
    for name in ("sweep", "couette", "fourier_cyl"):
        ps, desc = bench.workload(name, 2, "fp32")
        assert all(p["precision"] == 1 for p in ps) and "FP32" in desc
    ps, _ = bench.workload("sweep", 2, "fp64")
    assert all(p["precision"] == 0 for p in ps)
    cb = bench.cpu_baseline(bench.workload("couette", 1, "fp32")[0], 0.5)
    assert cb["value"] > 0 and cb["kind"] == "oracle" and cb["cores"] >= 1
    one = bench.cpu_baseline(bench.workload("couette", 1, "fp32")[0], 0.3, threads=1)
    assert one["cores"] == 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2 and "one GPU" in r.stderr
