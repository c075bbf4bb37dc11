"""Host-side pieces of bench.py (no GPU): workloads carry the storage precision, the CPU baseline
runs the FP64 oracle on them, more than one GPU is refused with a message, and the committed HBM
traffic measurement is reported only for the workload it was taken on."""
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


def test_traffic_only_for_the_measured_workload():
    """The counter measurement of the stage kernel is for the 256-instance sweep: the sweep's
    algorithmic bytes per stage launch (site-velocities x 8 bytes per value read or written x 3
    accesses per step averaged over the three stages: 32 / 3 B with FP32 storage, 64 / 3 B with
    FP64) get it while the kernel source is unchanged; any other workload gets None."""
    ps, _ = bench.workload("sweep", 256, "fp32")
    sv = sum(p["nr"] * 2 * p["q_radial"] * p["q_t1"] * p["q_t2"] for p in ps)
    for prec, fbytes in (("fp32", 4), ("fp64", 8)):
        b = sv * 8.0 * fbytes / 3
        t = bench.measured_traffic(prec, b)
        assert t is not None and t > b, prec
        assert bench.measured_traffic(prec, b * 0.5) is None
    assert bench.measured_traffic("fp64", 7603200 * 64 / 3) is None  # the paper's grid, FP64
