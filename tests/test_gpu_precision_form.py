"""The precision form at full size: 1080p, N in {4, 16, 64}, widths 64 and 128, FP32 / BF16 /
FP16 estimates checked against the FP64 oracle on a seeded subset of the frame's points (the
oracle draws the directions by the points' frame indices).  Prints the error table the precision
form reports; bounds as in the parity tests (rel-L2 of F_tl relative to |F_c|: 1e-5 FP32, 1e-2
16-bit) with per-point bounds beside them."""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import check_estimate_points, host, residual_prediction

pytestmark = pytest.mark.gpu
P = 1920 * 1080
BOUND = {"fp32": 1e-5, "bf16": 1e-2, "fp16": 1e-2}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


@pytest.fixture(scope="module")
def frame_points(nirc):
    pts = wl.make_points(3, P)
    return pts, nirc.Points.from_workload(pts)


@pytest.mark.parametrize("W", [64, 128])
@pytest.mark.parametrize("N", [4, 16, 64])
def test_precision_form_against_oracle_subset(nirc, frame_points, W, N):
    pts, dp = frame_points
    lobes = wl.make_lobes(3).packed()
    w = wl.make_weights(3, W)
    sel = np.sort(np.random.default_rng(4321 + N + W).choice(P, 1024, replace=False))
    sel = np.unique(np.concatenate([sel, np.arange(P - 8, P)]))
    sub = pts.subset(sel)
    dirs = oracle.sample_dirs(sub, N, 3, 0, ids=sel)
    o_tl, o_c, o_r = oracle.estimate(sub, lobes, w, W, N, 3, 0, dirs=dirs)
    y_r = residual_prediction(sub, w, W, N, 3, 0, dirs=dirs)
    line = [f"W={W:3d} N={N:2d}"]
    for name, prec in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
        m = nirc.Model(w, cfg=nirc.make_config(width=W, precision=prec), max_batch=0)
        tl, c, r = (host(t)[sel] for t in nirc.tlmc_estimate(m, dp, lobes, N, 3, 0, parts=True))
        e_tl = float(np.linalg.norm(tl - o_tl) / np.linalg.norm(o_c))
        e_c = float(np.linalg.norm(c - o_c) / np.linalg.norm(o_c))
        line.append(f"{name}: F_tl {e_tl:.2e} F_c {e_c:.2e}")
        assert e_tl <= BOUND[name] and e_c <= BOUND[name], (name, e_tl, e_c)
        check_estimate_points(f"{name} W={W} N={N}", tl, c, r, o_tl, o_c, o_r, y_r, name)
        del m
    print("precision form vs oracle subset | " + " | ".join(line), flush=True)
