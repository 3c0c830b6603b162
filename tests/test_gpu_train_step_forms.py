"""A training step (nirc_train_step: gradient partials, fixed-order reduction, then Adam with the
refresh of the kernels' weight copy and the step commit in one launch) gives, bit for bit, what
the separate calls give: the gradient (nirc_loss_grad), then Adam on it (nirc_adam_step)
(Sec. "Results": several Adam steps per frame).  The copy that Adam refreshes parameter by
parameter through the inverse packing map equals a full repack of the master weights, and a step
with a non-finite gradient leaves everything but the flags as it was."""
import numpy as np
import pytest
import torch

from paper_2412_04634_amd import workload as wl
from tests.common import host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def _state_equal(a, b):
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    for x, y in zip(a.get_adam(), b.get_adam()):
        np.testing.assert_array_equal(host(x), host(y))
    assert a.read_flags() == b.read_flags()
    assert a.read_loss_scale() == b.read_loss_scale()


@pytest.mark.parametrize("width", [64, 128])
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_train_step_equals_gradient_then_adam(nirc, prec, width):
    pts = wl.make_points(41, 1500)
    dp = nirc.Points.from_workload(pts)
    lobes = wl.make_lobes(41).packed()
    w0 = wl.make_weights(41, width)
    B = 3000   # several gradient blocks and a ragged last one
    cfg = nirc.make_config(width=width, precision=prec)
    a = nirc.Model(w0, cfg=cfg, max_batch=B)
    b = nirc.Model(w0, cfg=cfg, max_batch=B)
    for step in range(3):
        q, t = nirc.tlmc_train_batch(dp, lobes, B, 42, 0, step)
        la = torch.zeros(1, device="cuda")
        nirc.nirc_train_step(a, dp, q, t, loss=la)
        lb, g = nirc.nirc_loss_grad(b, dp, q, t)
        nirc.nirc_adam_step(b, g)
        torch.cuda.synchronize()
        assert host(la)[0] == host(lb)[0]
    _state_equal(a, b)
    # the refreshed copy is the one the kernels read: inference agrees too
    q, _ = nirc.tlmc_train_batch(dp, lobes, 500, 43, 0, 0)
    np.testing.assert_array_equal(host(nirc.nirc_infer(a, dp, q)), host(nirc.nirc_infer(b, dp, q)))
    # the copy refreshed parameter by parameter equals a full repack of the trained master weights
    c = nirc.Model(host(a.get_weights()), cfg=cfg, max_batch=0)
    np.testing.assert_array_equal(host(nirc.nirc_infer(c, dp, q)), host(nirc.nirc_infer(a, dp, q)))


@pytest.mark.parametrize("prec", [0, 1])
def test_train_step_with_a_non_finite_gradient_changes_nothing(nirc, prec):
    pts = wl.make_points(44, 1200)
    dp = nirc.Points.from_workload(pts)
    lobes = wl.make_lobes(44).packed()
    w0 = wl.make_weights(44, 64)
    B = 2048
    cfg = nirc.make_config(precision=prec)
    a = nirc.Model(w0, cfg=cfg, max_batch=B)
    b = nirc.Model(w0, cfg=cfg, max_batch=B)
    q, t = nirc.tlmc_train_batch(dp, lobes, B, 45, 0, 0)
    nirc.nirc_train_step(a, dp, q, t)
    nirc.nirc_train_step(b, dp, q, t)
    torch.cuda.synchronize()
    before = host(a.get_state()).copy()
    # one sample's target is NaN: every gradient sum it reaches is NaN, so the step is skipped
    q2, t2 = nirc.tlmc_train_batch(dp, lobes, B, 45, 0, 1)
    t2 = t2.clone()
    t2[B - 7, 1] = float("nan")
    nirc.nirc_train_step(a, dp, q2, t2)
    _, g = nirc.nirc_loss_grad(b, dp, q2, t2)
    nirc.nirc_adam_step(b, g)
    torch.cuda.synchronize()
    assert a.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD
    assert b.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD
    after = host(a.get_state())
    _state_equal(a, b)
    # nothing but the flags word moved: weights, moments, packed copies and the step count are
    # those before the step
    assert 1 <= int((after != before).sum()) <= 4, np.flatnonzero(after != before)
    # and the next finite step trains both alike
    q3, t3 = nirc.tlmc_train_batch(dp, lobes, B, 45, 0, 2)
    nirc.nirc_train_step(a, dp, q3, t3)
    _, g = nirc.nirc_loss_grad(b, dp, q3, t3)
    nirc.nirc_adam_step(b, g)
    _state_equal(a, b)
