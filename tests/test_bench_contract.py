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


def test_leaf_traffic_only_for_the_measured_source_and_configuration(monkeypatch):
    import hashlib
    src = os.path.join(ROOT, "paper_1011_3534_amd", "csrc", "leaf.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    table = dict(bench.PMC_TRAFFIC)
    key = next(iter(table["leaf"]))
    # counters taken on this very source: the figure is reported for their configuration only
    monkeypatch.setitem(bench.PMC_TRAFFIC, "src_sha256_16", sha)
    prec, leaf, n, tau, build = key
    t = bench.leaf_traffic(prec, leaf, n, tau, build)
    f, w = table["leaf"][key]
    assert t == (f * table["fetch_factor"] + w * table["write_factor"]) * 1024.0
    assert bench.leaf_traffic(prec, leaf, n, tau, "packed" if build == "view" else "view") is None
    assert bench.leaf_traffic(prec, leaf, n // 2, tau, build) is None
    # counters of another source: nothing is reported
    monkeypatch.setitem(bench.PMC_TRAFFIC, "src_sha256_16", "0" * 16)
    assert bench.leaf_traffic(prec, leaf, n, tau, build) is None
