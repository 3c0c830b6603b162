"""bench.py's command line on the CPU: more than one GPU is refused with a message (the hot path
runs on one GPU), the flop counts it reports follow the per-point formulas, and the locality
order it times the hash-grid estimate with is a permutation of neighbours."""
import json
import os
import subprocess
import sys

import numpy as np

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


def test_morton_order_is_a_locality_permutation():
    from paper_2412_04634_amd import workload as wl
    p = wl.make_points(5, 20000)
    o = wl.morton_order(p)
    assert np.array_equal(np.sort(o), np.arange(p.count))
    q = p.subset(o)
    step = lambda a: np.abs(np.diff(a.px)) + np.abs(np.diff(a.py)) + np.abs(np.diff(a.pz))
    # consecutive points are neighbours in the new order (a random order steps ~1.0 on average)
    assert step(q).mean() < 0.1 * step(p).mean()
    # each point keeps its values
    assert np.array_equal(q.px, p.px[o]) and np.array_equal(q.rough, p.rough[o])
