"""Host logic of bench.py (CPU only): the refusal of several GPUs, the
counter records the roofline's traffic is read from, and the consistency of
its equal-accuracy degrees."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
F32_STEP = "cheb_step_kernel<float, float, false, true, 7, false>"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stdout and "--gpus must be 1" in r.stdout


@pytest.mark.parametrize("workload", ["anderson3d_128^3_W16_longrange2", "anderson3d_64^3_periodic_W16"])
def test_counter_records_match_the_current_step_kernel(workload):
    """The benchmark's two workloads have a counter record, at the probe-block
    width the benchmark runs them with, for the current step sources (a change to the step kernel leaves `traffic` null until the
    counters are taken again); the record's bytes are the calibrated
    FETCH_SIZE and WRITE_SIZE (factors 2 and 1, KiB; the KiB figures are
    recorded to 0.1 KiB)."""
    rec, why = bench.counter_traffic(F32_STEP, workload, bench.WORKLOADS[workload][3])
    assert rec is not None, why
    assert rec["source"].startswith("profiles/") and os.path.exists(os.path.join(ROOT, rec["source"]))
    assert abs(rec["bytes"] - (2.0 * rec["fetch_kib"] + 1.0 * rec["write_kib"]) * 1024) <= 3 * 0.05 * 1024


def test_records_are_kept_per_block_width():
    """The large workload has records at probe blocks of 32 (the benchmark's
    setting) and 64, each found only under its own width; a record without
    a width is for 64."""
    w = "anderson3d_128^3_W16_longrange2"
    r32, _ = bench.counter_traffic(F32_STEP, w, 32)
    r64, _ = bench.counter_traffic(F32_STEP, w, 64)
    assert r32 is not None and r64 is not None and r32["bytes"] != r64["bytes"]
    assert bench.counter_traffic(F32_STEP, w, 128)[0] is None
    assert bench.counter_traffic(F32_STEP, "anderson3d_64^3_periodic_W16")[0] is not None


def test_unknown_kernel_or_workload_has_no_record():
    rec, why = bench.counter_traffic(F32_STEP, "no_such_workload")
    assert rec is None and "no counter record" in why
    rec, why = bench.counter_traffic("no_such_kernel<>", "anderson3d_64^3_periodic_W16")
    assert rec is None


def test_equal_accuracy_degrees_are_consistent():
    for j, n in ((bench.M_FP64_JACKSON, bench.M_FP32_NONE), (bench.M_LARGE_FP64_JACKSON, bench.M_LARGE_FP32_NONE),
                 (bench.M_BATCHED_FP64_JACKSON, bench.M_BATCHED_FP32_NONE)):
        assert 0 < n < j
    for m in (bench.M_FP32_LEARNED, bench.M_LARGE_FP32_LEARNED):
        assert 0 < m <= 127  # the network's widest input
    assert bench.M_BATCHED_FP32_LEARNED is None or bench.M_BATCHED_FP32_LEARNED <= 127
