"""bench.py's command line on the CPU: more than one GPU is refused with a message (the hot path
runs on one GPU), and the flop counts it reports follow the per-point formulas."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_algorithmic_flops():
    # surface projection once per point + (N + 1) queries of 48 W + 3 W^2 + 3 W multiply-adds
    assert bench.algorithmic_flops_estimate(2073600, 16, 64) == 1126180454400.0
    assert bench.algorithmic_flops_estimate(1, 0, 64) == 2 * 112 * 64 + 2 * (48 * 64 + 3 * 64 * 64 + 3 * 64)
    w = 128
    assert bench.algorithmic_flops_train(1, w) == 2 * (160 * w + 3 * w * w + 3 * w) * 2 + 2 * (3 * w * w + 3 * w)


def test_cpu_baseline_leg_runs():
    # the oracle leg of the bench line on a tiny frame (small time targets): keys and units
    from paper_2412_04634_amd import workload as wl
    pts = wl.make_points(3, 2048)
    lob = wl.make_lobes(3).packed()
    w0 = wl.make_weights(3, 64)
    r = bench.cpu_baseline(pts, lambda f: lob, w0, 64, 4, 256, 1, target_s=0.05, target_1core_s=0.05)
    assert r["kind"] == "oracle" and r["unit"] == "queries/s" and r["value"] > 0 and r["cores"] >= 1
    assert r["one_core"]["cores"] == 1 and r["one_core"]["value"] > 0
