"""Dynamic loss scaling of FP16 models: an overflowing scale (forced from the host by a huge
starting value) makes steps non-finite; each such step is skipped and halves the scale until
steps go through, and then training continues exactly as a model started at the backed-off
scale; 1000 finite steps in a row double it; the training state carries it; BF16 keeps its
static scale."""
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


def _scene(nirc, seed, P=2000):
    pts = wl.make_points(seed, P)
    return nirc.Points.from_workload(pts), wl.make_lobes(seed).packed(), wl.make_weights(seed, 64)


def test_fp16_overflow_backs_off_then_trains_like_the_backed_off_model(nirc):
    dp, lobes, w0 = _scene(nirc, 91)
    B = 4096
    a = nirc.Model(w0, cfg=nirc.make_config(precision=2, loss_scale=2.0 ** 22), max_batch=B)
    batches = [nirc.tlmc_train_batch(dp, lobes, B, 92, 0, s) for s in range(40)]
    skipped = 0
    for q, t in batches:
        nirc.nirc_train_step(a, dp, q, t)
        _, _, step = a.get_adam()
        if int(step.item()) > 0:
            break
        skipped += 1
    assert 1 <= skipped < 30, skipped
    assert a.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD
    assert a.read_loss_scale() == 2.0 ** (22 - skipped)
    # a model started at the backed-off scale, given the batches from the first one that went
    # through, ends bit for bit alike
    b = nirc.Model(w0, cfg=nirc.make_config(precision=2, loss_scale=2.0 ** (22 - skipped)), max_batch=B)
    for q, t in batches[skipped:skipped + 1]:
        nirc.nirc_train_step(b, dp, q, t)
    for q, t in batches[skipped + 1:skipped + 6]:
        nirc.nirc_train_step(a, dp, q, t)
        nirc.nirc_train_step(b, dp, q, t)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    for x, y in zip(a.get_adam(), b.get_adam()):
        np.testing.assert_array_equal(host(x), host(y))
    # (a later overflow backs both off alike)
    assert a.read_loss_scale() == b.read_loss_scale() <= 2.0 ** (22 - skipped)
    # the state blob carries the scale
    c = nirc.Model(w0, cfg=nirc.make_config(precision=2, loss_scale=1.0), max_batch=B)
    c.set_state(a.get_state())
    assert c.read_loss_scale() == a.read_loss_scale()


def test_fp16_scale_grows_after_a_run_of_finite_steps(nirc):
    dp, lobes, w0 = _scene(nirc, 93, P=500)
    B = 64
    m = nirc.Model(w0, cfg=nirc.make_config(precision=2, loss_scale=1.0), max_batch=B)
    q, t = nirc.tlmc_train_batch(dp, lobes, B, 94, 0, 0)
    for _ in range(999):
        nirc.nirc_train_step(m, dp, q, t)
    assert m.read_loss_scale() == 1.0
    nirc.nirc_train_step(m, dp, q, t)
    assert m.read_loss_scale() == 2.0
    assert m.read_flags() == 0
    _, _, step = m.get_adam()
    assert int(step.item()) == 1000


def test_bf16_scale_is_static(nirc):
    dp, lobes, w0 = _scene(nirc, 95, P=500)
    B = 256
    m = nirc.Model(w0, cfg=nirc.make_config(precision=1, loss_scale=4.0), max_batch=B)
    q, t = nirc.tlmc_train_batch(dp, lobes, B, 96, 0, 0)
    t[3, 0] = float("nan")
    nirc.nirc_train_step(m, dp, q, t)
    assert m.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD
    assert m.read_loss_scale() == 4.0
