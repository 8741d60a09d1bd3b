"""Host-side pieces of bench.py (no GPU): the CPU baseline and the --gpus contract."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cpu_baseline_small():
    import bench
    from workloads import config_c1

    r = bench.cpu_baseline(config_c1(), 55, 16)
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["unit"] == "DOF-shift-solves/s"
    assert r["value"] > 0 and "extrapolated" in r["sample"]


def test_multi_gpu_request_exits_with_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_traffic_record_matches_kernel_source_or_is_dropped():
    import hashlib

    import bench

    with open(os.path.join(ROOT, bench.TRAFFIC_SOURCE), "rb") as f:
        current = hashlib.sha256(f.read()).hexdigest()
    t = bench._traffic("ends_fwd", "blocked")
    assert (t is None) == (current != bench.TRAFFIC_SHA256)
