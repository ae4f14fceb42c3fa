"""Host-side parts of bench.py's contract (no GPU): it refuses more than one
GPU with a message, and the leaf traffic figure is only reported for the
kernel source and configuration the counters were taken on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_leaf_traffic_only_for_the_measured_source_and_configuration():
    t = bench.leaf_traffic("f16x3", 64, 8192, 1e-6, "view")
    assert t is not None and 0.5e9 < t < 1.5e9          # reads beyond L2 + writes, bytes per launch
    assert bench.leaf_traffic("f16x3", 64, 8192, 1e-6, "packed") is None
    assert bench.leaf_traffic("f16x3", 64, 4096, 1e-6, "view") is None
    assert bench.leaf_traffic("bf16x3", 64, 8192, 1e-6, "view") is None
