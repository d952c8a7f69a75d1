"""CPU checks of the benchmark's contract: one GPU only, and counter traffic reported only when the
stored profiler counts were taken on the current kernel source."""
import json
import os
import subprocess
import sys

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
