"""bench.py plumbing that runs without a GPU: the single-GPU contract and the
rule for quoting the committed HBM-traffic record of the benchmarked kernel."""
import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_traffic_is_reported_only_for_the_current_kernel_source(tmp_path, monkeypatch):
    """The bench quotes HBM traffic from a committed counter record only while
    that record was taken on the current step-kernel source, compiler flags,
    kernel and workload; any change to the kernels turns the figure into null
    until counters are taken again."""
    wl, k = bench.DEFAULT_WORKLOAD, "step_kernel"
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    assert bench.stored_traffic(k, wl) is None  # no record
    rec = {"workload": wl, "kernel": k, "kernel_source_sha256_16": bench.kernel_source_hash(),
           "hbm_bytes_per_launch": 123456789}
    path = tmp_path / f"{k}_{wl}_traffic.json"
    path.write_text(json.dumps(rec))
    assert bench.stored_traffic(k, wl) == 123456789
    assert bench.stored_traffic("step_pair_kernel", wl) is None  # another kernel
    rec["kernel_source_sha256_16"] = "0" * 16
    path.write_text(json.dumps(rec))
    assert bench.stored_traffic(k, wl) is None
    assert bench.stored_traffic(k, "no_such_workload") is None
