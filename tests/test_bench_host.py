"""Host-side checks of bench.py: the single-GPU contract and the work model."""

import subprocess
import sys

import bench


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, "bench.py", "--gpus", "2"], capture_output=True, text=True,
                       cwd=bench.ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_stage_work_is_sum_of_kernel_parts():
    for N in range(0, 9):
        Fs, _ = bench.stage_work(N)
        Ft, _ = bench.kernel_work("trace", N)
        Fst, _ = bench.kernel_work("stage", N)
        assert Fs == Ft + Fst


def test_traffic_record_requires_matching_sources():
    assert bench.recorded_traffic("stage", "no such workload") is None
    v = bench.recorded_traffic("stage", "k1d=40 N=4 fp64 fused")
    assert v is None or v > 0
