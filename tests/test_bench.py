"""CPU checks of the benchmark's contract: one GPU only, a roofline on bytes the kernels move, and counter
traffic reported only when the stored profiler counts were taken on the current kernel source."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_stored_traffic_requires_the_current_kernel_source(tmp_path):
    rec = {"kernels_sha256": bench.kernels_digest(), "fetch_bytes_per_iteration": 3.0e9,
           "write_bytes_per_iteration": 1.0e9, "launches_per_iteration": 13}
    good = tmp_path / "good.json"
    good.write_text(json.dumps({"k_level/large/fp32": rec}))
    assert bench.stored_traffic("k_level", "large", "fp32", 13, path=str(good)) == 4.0e9 / 13
    # another workload, precision or kernel has no record
    assert bench.stored_traffic("k_level", "large", "fp64", 13, path=str(good)) is None
    assert bench.stored_traffic("k_forward", "large", "fp32", 12, path=str(good)) is None
    stale = tmp_path / "stale.json"
    stale.write_text(json.dumps({"k_level/large/fp32": dict(rec, kernels_sha256="0" * 64)}))
    assert bench.stored_traffic("k_level", "large", "fp32", 13, path=str(stale)) is None
    assert bench.stored_traffic("k_level", "large", "fp32", 13, path=str(tmp_path / "missing.json")) is None


def test_committed_profiles_name_their_kernel_source():
    """Every record of the committed counter summary carries the digest it was taken on and the
    command that produced it."""
    data = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))
    assert data
    for key, rec in data.items():
        assert len(rec["kernels_sha256"]) == 64, key
        assert "rocprofv3" in rec["command"], key
        assert rec["fetch_bytes_per_iteration"] > 0 and rec["write_bytes_per_iteration"] > 0, key


def test_roofline_uses_design_bytes_and_rejects_impossible_rates():
    kernels = [dict(name="k_forward", launches_per_iteration=12, bytes_per_iteration=1.2e9,
                    method_bytes_per_iteration=4.1e9, ms_per_iteration=0.30),
               dict(name="k_level", launches_per_iteration=13, bytes_per_iteration=2.94e9,
                    method_bytes_per_iteration=7.5e9, ms_per_iteration=0.79)]
    r = bench.roofline_record(kernels, lambda name, nl: 3.39e9 / nl)
    assert r["kernel"] == "k_level"
    per_launch_ms = 0.79 / 13
    assert abs(r["achieved"] - 2.94e9 / 13 / (per_launch_ms * 1e-3) / 1e9) < 1e-6
    assert abs(r["frac"] - r["achieved"] / 8000.0) < 1e-12 and 0 < r["frac"] <= 1
    assert abs(r["traffic_over_design"] - 3.39 / 2.94) < 1e-9
    # the method's figures stay informational: here they would exceed the peak
    assert r["achieved_method_bytes"] > 8000.0
    with pytest.raises(ValueError):
        bench.physical_rate(9.0e9, 1.0)
    assert abs(bench.physical_rate(4.0e9, 1.0) - 4000.0) < 1e-9


def test_recorded_benchmark_lines_are_physical():
    """Every benchmark record the driver kept: the design bytes of one iteration over its measured
    time stay within the HBM peak."""
    import glob
    for path in sorted(glob.glob(os.path.join(ROOT, "BENCH_r*.json"))):
        rec = json.load(open(path))
        line = rec.get("parsed") or rec
        if not line or "design_bytes_per_iteration" not in line or not line.get("ms_per_step"):
            continue
        bench.physical_rate(line["design_bytes_per_iteration"], line["ms_per_step"])
