"""The benchmark's host-side bookkeeping (no GPU): the algorithmic flop count
of the network, the --gpus guard, and that the stored HBM traffic of the
network kernel was measured on the kernel sources in the tree."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_flops_per_eval():
    # 6-256x6-1: 4 (D-1) H^2 + 22 H = 1,316,352 (forward + source gradient)
    assert bench.flops_per_eval(256, 6) == 1_316_352
    assert bench.flops_per_eval(32, 3) == 4 * 2 * 32 * 32 + 22 * 32


def test_stored_traffic_matches_the_kernel_sources():
    t = bench.NETWORK_TRAFFIC
    got = bench.network_traffic(t["rows"], t["variant"])
    assert got == t["fetch_bytes"] + t["write_bytes"], \
        "network kernel sources changed: retake FETCH_SIZE / WRITE_SIZE"
    assert bench.network_traffic(t["rows"] + 1, t["variant"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0 and "one GPU" in (r.stdout + r.stderr)
