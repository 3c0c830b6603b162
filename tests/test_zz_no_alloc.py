"""nirc_train_step_static: the training step for callers that cannot allocate, on the library's
static device scratch, against nirc_train_step on a model with its own workspace.  Two calls in a
row, the second with a smaller batch; both models must end bit for bit alike."""
import numpy as np
import pytest
import torch

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


def _state(nirc, model):
    m, v, step = model.get_adam()
    return [host(model.get_weights()), host(m), host(v), int(step.item())]


@pytest.mark.parametrize("width,prec,loss", [(64, "fp32", 0), (64, "bf16", 0), (64, "fp16", 0), (128, "fp32", 0),
                                             (128, "bf16", 0), (64, "fp32", 2), (64, "bf16", 1)])
def test_static_train_step_matches_workspace_step(nirc, width, prec, loss):
    print(f"static train step W={width} {prec} loss={loss}", flush=True)
    P = 5000
    pts = wl.make_points(81, P)
    lobes = wl.make_lobes(81).packed()
    w0 = wl.make_weights(81, width)
    dp = nirc.Points.from_workload(pts)
    cfg = nirc.make_config(width=width, precision=PRECS[prec], loss=loss,
                           loss_scale=(128.0 if prec == "fp16" else 1.0))
    a = nirc.Model(w0, cfg=cfg, max_batch=nirc.NIRC_STATIC_MAX_BATCH)
    b = nirc.Model(w0, cfg=cfg, max_batch=0)   # no workspace at all
    for call, B in enumerate([nirc.NIRC_STATIC_MAX_BATCH, 333]):
        q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 82, 0, call)
        la = torch.full((1,), -1.0, device="cuda")
        lb = torch.full((1,), -2.0, device="cuda")
        nirc.nirc_train_step(a, dp, q, tgt, la)
        nirc.nirc_train_step_static(b, dp, q, tgt, lb)
        torch.cuda.synchronize()
        sa, sb = _state(nirc, a), _state(nirc, b)
        for x, y in zip(sa[:3], sb[:3]):
            np.testing.assert_array_equal(x, y)
        assert sa[3] == sb[3] == call + 1
        assert la.item() == lb.item() and np.isfinite(la.item())
        assert a.read_flags() == 0 and b.read_flags() == 0
    # the model without workspace cannot take the ordinary step; the static one refuses batches
    # above its maximum before enqueuing anything
    q, tgt = nirc.tlmc_train_batch(dp, lobes, nirc.NIRC_STATIC_MAX_BATCH + 1, 82, 0, 5)
    with pytest.raises(nirc.NircError):
        nirc.nirc_train_step(b, dp, q, tgt)
    before = _state(nirc, b)
    with pytest.raises(nirc.NircError):
        nirc.nirc_train_step_static(b, dp, q, tgt)
    after = _state(nirc, b)
    for x, y in zip(before[:3], after[:3]):
        np.testing.assert_array_equal(x, y)
    assert before[3] == after[3]


def test_static_train_step_on_two_models_in_turn(nirc):
    # the scratch keeps the last call's contents; a step on another model (another width) in
    # between must not change what the next step computes
    P, B = 3000, 1000
    pts = wl.make_points(83, P)
    lobes = wl.make_lobes(83).packed()
    dp = nirc.Points.from_workload(pts)
    cfg64, cfg128 = nirc.make_config(width=64), nirc.make_config(width=128, precision=1)
    a = nirc.Model(wl.make_weights(83, 64), cfg=cfg64, max_batch=B)
    b = nirc.Model(wl.make_weights(83, 64), cfg=cfg64, max_batch=0)
    c = nirc.Model(wl.make_weights(84, 128), cfg=cfg128, max_batch=0)
    for k in range(3):
        q, tgt = nirc.tlmc_train_batch(dp, lobes, B - 100 * k, 85, 0, k)
        nirc.nirc_train_step(a, dp, q, tgt)
        nirc.nirc_train_step_static(c, dp, q, tgt)
        nirc.nirc_train_step_static(b, dp, q, tgt)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    assert b.read_flags() == 0 and c.read_flags() == 0
