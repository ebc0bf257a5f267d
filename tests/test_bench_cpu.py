"""bench.py plumbing that runs without a GPU: the single-GPU contract and the
committed HBM-traffic record of the benchmarked kernel."""
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


def test_traffic_record_matches_the_current_kernel_source():
    """The counters under profiles/ were taken on this step-kernel source; a
    change to the kernels without a new counter run would turn the bench's
    traffic figure into null."""
    wl = bench.DEFAULT_WORKLOAD
    path = os.path.join(ROOT, "profiles", f"step_kernel_{wl}_traffic.json")
    with open(path) as f:
        rec = json.load(f)
    assert rec["kernel_source_sha256_16"] == bench.kernel_source_hash()
    t = bench.stored_traffic(wl, 0)
    assert t is not None and t > rec["algorithmic_bytes_per_launch"]
    assert bench.stored_traffic("no_such_workload", 0) is None
