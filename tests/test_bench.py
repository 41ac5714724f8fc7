"""The benchmark's contract on the CPU: one-GPU guard and the roofline
arithmetic of the dominant kernel from library phase timings."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_kernel_roofline_per_launch_figures():
    n, n_bins, steps = 1_600_000_000, 86_400_000, 10
    phases = {"lookup_ms": 0.0, "stage1_ms": 89.0, "index_ms": 2.0, "stage2_ms": 26.0,
              "far_ms": 0.1, "calls": steps, "stage1_launches": steps}
    r = bench.kernel_roofline(phases, n, n_bins, steps, "some other workload")
    assert r["kernel"] == "k_stage1"
    assert r["alg_bytes_per_launch"] == 21 * n      # one launch per step
    assert abs(r["launch_ms"] - 8.9) < 1e-9
    assert abs(r["achieved"] - 21 * n / 8.9e-3 / 1e9) < 1e-6
    assert r["frac"] == r["achieved"] / 8000.0
    assert r["traffic"] is None                     # counters belong to another workload
    # a separate lookup pass: stage 1 reads 13 B/session, the pass 9 B/session
    phases2 = dict(phases, lookup_ms=200.0)
    r2 = bench.kernel_roofline(phases2, n, n_bins, steps, "w")
    assert r2["kernel"].startswith("k_pass") and r2["alg_bytes_per_launch"] == 9 * n
    # two launches per step (sessions beyond 2^31 are split in pieces)
    phases3 = dict(phases, stage1_launches=2 * steps)
    r3 = bench.kernel_roofline(phases3, n, n_bins, steps, "w")
    assert r3["alg_bytes_per_launch"] == 21 * n / 2 and abs(r3["launch_ms"] - 4.45) < 1e-9
    assert bench.kernel_roofline(None, n, n_bins, steps, "w") is None
