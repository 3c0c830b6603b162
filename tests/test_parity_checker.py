"""The per-point parity checks used by the GPU tests, exercised on the CPU with oracle values:
an exact result passes, and corrupting one point of a few thousand by 1e-4 (FP32 bound) or 1 %
(16-bit bounds) fails them, where the rel-L2 over the array alone would let it through."""
import numpy as np
import pytest

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import POINT_TOL, QUERY_TOL, check_estimate_points, check_query_points, rel_l2, residual_prediction

W = 64


@pytest.fixture(scope="module")
def est():
    P, N, seed, frame = 4096, 8, 5, 1
    pts = wl.make_points(90, P)
    lob = wl.make_lobes(90).packed()
    w0 = wl.make_weights(90, W)
    tl, c, r = oracle.estimate(pts, lob, w0, W, N, seed, frame)
    y_r = residual_prediction(pts, w0, W, N, seed, frame)
    return tl, c, r, y_r


def _scale(c, y_r, p):
    return float(np.linalg.norm(c[p]) + np.linalg.norm(y_r[p]))


@pytest.mark.parametrize("prec,size", [("fp32", 1e-4), ("bf16", 1e-2), ("fp16", 1e-2)])
@pytest.mark.parametrize("part", ["c", "r", "tl"])
def test_one_corrupted_point_fails(est, prec, size, part):
    tl, c, r, y_r = est
    check_estimate_points("exact", tl, c, r, tl, c, r, y_r, prec)
    p = 1234
    got = {"tl": tl.copy(), "c": c.copy(), "r": r.copy()}
    # one point moved by `size` of its own scale (F_c: of |F_c,p|), along the first channel
    s = float(np.linalg.norm(c[p])) if part == "c" else _scale(c, y_r, p)
    got[part][p, 0] += size * s
    # the array norms alone miss it ...
    norm_tol = 1e-5 if prec == "fp32" else 1e-2
    assert np.linalg.norm(got[part] - {"tl": tl, "c": c, "r": r}[part]) <= norm_tol * np.linalg.norm(c)
    # ... the per-point bound does not
    assert size > POINT_TOL[prec]
    with pytest.raises(AssertionError):
        check_estimate_points("corrupted", got["tl"], got["c"], got["r"], tl, c, r, y_r, prec)


@pytest.mark.parametrize("prec,size", [("fp32", 1e-4), ("fp16", 1e-2)])
def test_one_corrupted_query_fails(prec, size):
    P, Q = 300, 4099
    pts = wl.make_points(91, P)
    w0 = wl.make_weights(91, W)
    rng = np.random.default_rng(3)
    idx = rng.integers(0, P, Q).astype(np.int32)
    d = rng.normal(size=(Q, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ref = oracle.infer(pts, idx, d, w0, W)
    check_query_points("exact", ref, ref, prec)
    got = ref.copy()
    got[77, 1] += size * np.linalg.norm(ref[77])
    assert rel_l2(got, ref) <= (1e-5 if prec == "fp32" else 1e-2)
    assert size > QUERY_TOL[prec]
    with pytest.raises(AssertionError):
        check_query_points("corrupted", got, ref, prec)
