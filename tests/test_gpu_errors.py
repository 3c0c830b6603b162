"""Errors found on the device: a query naming a point index outside the point set.

The kernels never read out of bounds for such an index; they raise NIRC_FLAG_BAD_POINT_INDEX in
the model's flags, a training step that meets one is skipped, and nirc_encode writes NaN features
for the query.  The other queries of the call are unaffected."""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import host

pytestmark = pytest.mark.gpu
PRECS = {"fp32": 0, "bf16": 1, "fp16": 2}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def _queries(nirc, P, Q, bad_at, bad_value, seed):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(Q, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    idx = rng.integers(0, P, Q).astype(np.int32)
    good = nirc.Queries.from_dirs(torch.from_numpy(d.astype(np.float32)).cuda(), torch.from_numpy(idx).cuda())
    idx_bad = idx.copy()
    idx_bad[bad_at] = bad_value
    bad = nirc.Queries.from_dirs(torch.from_numpy(d.astype(np.float32)).cuda(), torch.from_numpy(idx_bad).cuda())
    return good, bad


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("bad_value", [-1, 300, 2 ** 31 - 1])
def test_infer_bad_point_index_raises_flag(nirc, prec, bad_value):
    print(f"bad index infer {prec} {bad_value}", flush=True)
    P, Q = 300, 100
    pts = wl.make_points(61, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(wl.make_weights(61, 64), cfg=nirc.make_config(precision=PRECS[prec]), max_batch=0)
    good, bad = _queries(nirc, P, Q, 37, bad_value, 62)
    y_good = host(nirc.nirc_infer(model, dp, good))
    assert model.read_flags() == 0
    y_bad = host(nirc.nirc_infer(model, dp, bad))
    assert model.read_flags() & nirc.NIRC_FLAG_BAD_POINT_INDEX
    keep = np.arange(Q) != 37
    np.testing.assert_array_equal(y_bad[keep], y_good[keep])
    model.clear_flags()
    assert model.read_flags() == 0


def test_encode_bad_point_index_gives_nan(nirc):
    P, Q = 300, 50
    pts = wl.make_points(63, P)
    dp = nirc.Points.from_workload(pts)
    good, bad = _queries(nirc, P, Q, 11, P, 64)
    f_good = host(nirc.nirc_encode(dp, good))
    f_bad = host(nirc.nirc_encode(dp, bad))
    assert np.all(np.isfinite(f_good))
    keep = np.arange(Q) != 11
    np.testing.assert_array_equal(f_bad[keep], f_good[keep])
    # the point-dependent inputs (x, n, roughness) have NaN features; the direction's are defined
    row = f_bad[11].reshape(10, 16)
    assert np.all(np.isnan(row[[0, 1, 2, 6, 7, 8, 9]]))


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_train_step_with_bad_point_index_is_skipped(nirc, prec):
    print(f"bad index train {prec}", flush=True)
    P, B = 400, 256
    pts = wl.make_points(65, P)
    lobes = wl.make_lobes(65).packed()
    w0 = wl.make_weights(65, 64)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 66, 0, 0)
    q.point[200] = P + 5
    nirc.nirc_train_step(model, dp, q, tgt)
    f = model.read_flags()
    assert f & nirc.NIRC_FLAG_BAD_POINT_INDEX and not f & nirc.NIRC_FLAG_NONFINITE_GRAD, f
    np.testing.assert_array_equal(host(model.get_weights()), w0.astype(np.float64))
    _, _, step = model.get_adam()
    assert int(step.item()) == 0
    # the standalone gradient reports it in the sticky flags as well
    model.clear_flags()
    nirc.nirc_loss_grad(model, dp, q, tgt)
    assert model.read_flags() & nirc.NIRC_FLAG_BAD_POINT_INDEX
    # with the index repaired the step goes through
    model.clear_flags()
    q.point[200] = 3
    nirc.nirc_train_step(model, dp, q, tgt)
    assert model.read_flags() == 0
    _, _, step = model.get_adam()
    assert int(step.item()) == 1


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hash_bad_point_index(nirc, prec):
    P, B = 400, 128
    grid = (10, 4, 1.5)
    pts = wl.make_points(67, P)
    lobes = wl.make_lobes(67).packed()
    w = wl.make_hash_weights(67, 64, 2 * oracle.hash_entries(grid), 0.5)
    dp = nirc.Points.from_workload(pts)
    model = nirc.HashModel(w, cfg=nirc.make_config(precision=PRECS[prec]), grid=nirc.make_hash_grid(*grid),
                           max_batch=B)
    good, bad = _queries(nirc, P, 64, 5, -7, 68)
    y_good = host(nirc.nirc_hash_infer(model, dp, good))
    assert model.read_flags() == 0
    y_bad = host(nirc.nirc_hash_infer(model, dp, bad))
    assert model.read_flags() & nirc.NIRC_FLAG_BAD_POINT_INDEX
    keep = np.arange(64) != 5
    np.testing.assert_array_equal(y_bad[keep], y_good[keep])
    # a training step on a fresh model with one bad index is skipped
    m2 = nirc.HashModel(w, cfg=nirc.make_config(precision=PRECS[prec]), grid=nirc.make_hash_grid(*grid),
                        max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 69, 0, 0)
    q.point[17] = P
    nirc.nirc_hash_train_step(m2, dp, q, tgt)
    f = m2.read_flags()
    assert f & nirc.NIRC_FLAG_BAD_POINT_INDEX and not f & nirc.NIRC_FLAG_NONFINITE_GRAD, f
    np.testing.assert_array_equal(host(m2.get_weights()), w.astype(np.float64))
