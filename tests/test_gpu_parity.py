"""Parity of the HIP path with the FP64 oracle on the same seeded inputs (needs the GPU).

Every input of the oracle is its own: the seeded scene, the oracle's own sampled directions and
training samples (passed to the GPU as FP32 query buffers where a call takes queries).

Tolerances (FP32 arithmetic on the GPU against FP64):
  * Philox words and training point indices: bit-exact;
  * directions: DIR_TOL absolute (FP32 rounding of the sampling map, a few ulp);
  * features: 1e-6 absolute;
  * cache outputs and loss on the same queries: relative L2 <= 1e-5;
  * the fused estimator (directions sampled inside the kernel, against the oracle's FP64
    directions): F_c relative L2 <= 1e-5, and F_tl, F_r within EST_TOL = 1e-5 of the norm of
    F_c.  A direction error delta moves the highest-frequency features by 2^7 pi delta and a
    lobe of sharpness kappa <= 50 by kappa delta; the oracle alone, fed directions perturbed by
    2e-7, moves F_r by 3.4e-6 of |F_c|, so directions within DIR_TOL = 3e-7 keep F_r and F_tl
    inside 1e-5 of |F_c| together with the FP32 rounding of the network;
  * gradients: relative L2 <= 1e-5.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import (Samples, check_estimate_points, check_query_points, host, oracle_dirs32, rel_l2,
                          residual_prediction)

pytestmark = pytest.mark.gpu

W = 64
DIR_TOL = 3e-7
EST_TOL = 1e-5


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def say(*a):
    print(*a, flush=True)


def scene(seed, P):
    pts = wl.make_points(seed, P)
    return pts, wl.make_lobes(seed).packed(), wl.make_weights(seed, W)


# ------------------------------------------------------------------------------------------

@pytest.mark.parametrize("P,N", [(1, 1), (17, 3), (256, 8), (1000, 16)])
def test_sample_dirs_match_oracle(nirc, P, N):
    say(f"sample_dirs P={P} N={N}")
    pts, _, _ = scene(3, P)
    dp = nirc.Points.from_workload(pts)
    seed, frame = 0xDEADBEEF12, 5
    d = host(nirc.tlmc_sample_dirs(dp, N, seed, frame))
    ref = oracle.sample_dirs(pts, N, seed, frame)
    err = np.abs(d - ref).max()
    say(f"  max direction error {err:.2e}")
    assert err <= DIR_TOL


def test_encode_matches_oracle(nirc):
    say("encode")
    pts, _, _ = scene(4, 300)
    dp = nirc.Points.from_workload(pts)
    dirs = oracle_dirs32(pts, 2, 9, 0)
    idx = torch.arange(300, device="cuda", dtype=torch.int32).repeat_interleave(3)
    q = nirc.Queries.from_dirs(torch.from_numpy(dirs).cuda(), idx)
    f = host(nirc.nirc_encode(dp, q))
    ref = oracle.encode(pts, idx.cpu().numpy(), dirs.astype(np.float64))
    assert np.abs(f - ref).max() <= 1e-6
    # exact special values: v = 0, 1/2, 1
    sp = wl.Points(*[np.array([0.0, 0.5, 1.0], np.float32) for _ in range(7)])
    spd = nirc.Points.from_workload(sp)
    dd = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5], [1.0, 1.0, 1.0]], np.float32)
    fe = host(nirc.nirc_encode(spd, nirc.Queries.from_dirs(torch.from_numpy(dd).cuda())))
    fo = oracle.encode(sp, None, dd.astype(np.float64))
    assert np.abs(fe - fo).max() <= 1e-7


@pytest.mark.parametrize("Q", [0, 1, 15, 16, 1000, 4099])
def test_infer_matches_oracle(nirc, Q):
    say(f"infer Q={Q}")
    P = 300
    pts, _, w0 = scene(5, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=0)
    g = torch.Generator().manual_seed(Q)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g, dtype=torch.float64)
    d = (d / d.norm(dim=1, keepdim=True).clamp_min(1e-9)).float()
    q = nirc.Queries.from_dirs(d.cuda(), idx.cuda())
    y = host(nirc.nirc_infer(model, dp, q))
    if Q == 0:
        assert y.shape == (0, 3)
        return
    ref = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0, W)
    assert rel_l2(y, ref) <= 1e-5
    check_query_points(f"infer Q={Q}", y, ref, "fp32")


def check_estimate(tl, c, r, o_tl, o_c, o_r, y_r=None):
    e_c = rel_l2(c, o_c)
    e_tl = np.linalg.norm(tl - o_tl) / np.linalg.norm(o_c)
    e_r = np.linalg.norm(r - o_r) / np.linalg.norm(o_c)
    say(f"  F_c rel-L2 {e_c:.2e}; F_tl, F_r error / |F_c| {e_tl:.2e}, {e_r:.2e}")
    assert e_c <= 1e-5
    assert e_tl <= EST_TOL
    # F_r = L - y can cancel: its error is bounded relative to the cache prediction's scale
    assert e_r <= EST_TOL
    if y_r is not None:
        check_estimate_points("per point", tl, c, r, o_tl, o_c, o_r, y_r, "fp32")


@pytest.mark.parametrize("P,N", [(1, 1), (17, 3), (2048, 8), (4096, 8), (1000, 16), (333, 24), (100, 64),
                                 (4001, 5), (1003, 1)])
def test_estimate_matches_oracle(nirc, P, N):
    say(f"estimate P={P} N={N}")
    pts, lobes, w0 = scene(6, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=0)
    seed, frame = 77, 2
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lobes, N, seed, frame, parts=True))
    o_tl, o_c, o_r = oracle.estimate(pts, lobes, w0, W, N, seed, frame)
    check_estimate(tl, c, r, o_tl, o_c, o_r, residual_prediction(pts, w0, W, N, seed, frame))
    np.testing.assert_array_equal(tl, host(nirc.tlmc_estimate(model, dp, lobes, N, seed, frame)))


def test_estimate_zero_output_layer_and_empty(nirc):
    say("estimate special cases")
    P, N = 100, 4
    pts, lobes, w0 = scene(8, P)
    w = w0.copy()
    w[-3 * W:] = 0.0
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w, max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lobes, N, 3, 0, parts=True))
    assert np.all(c == 1.0)
    # y = 1 everywhere, so F_tl = L(x, w_r): the field at the oracle's residual directions
    L = oracle.field(lobes, pts, None, oracle.sample_dirs(pts, N, 3, 0)[:, N, :])
    assert np.linalg.norm(tl - L) <= EST_TOL * np.linalg.norm(c)
    empty = nirc.Points([torch.zeros(0, device="cuda") for _ in range(7)])
    out = nirc.tlmc_estimate(model, empty, lobes, N, 3, 0)
    assert out.shape == (0, 3)


def test_train_batch_matches_oracle(nirc):
    say("train_batch")
    P, B = 5000, 4099
    pts, lobes, _ = scene(9, P)
    dp = nirc.Points.from_workload(pts)
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 11, 4, 3)
    idx, d, t = oracle.train_batch(pts, lobes, B, 11, 4, 3)
    np.testing.assert_array_equal(q.point.cpu().numpy(), idx)
    gd = np.stack([host(q.wx), host(q.wy), host(q.wz)], 1)
    assert np.abs(gd - d).max() <= DIR_TOL
    # targets: the field at directions within DIR_TOL, lobes of sharpness <= 50
    e_t = rel_l2(host(tgt), t)
    say(f"  target rel-L2 {e_t:.2e}")
    assert e_t <= EST_TOL


@pytest.mark.parametrize("B", [1, 65, 1000, 4096])
def test_loss_grad_matches_oracle(nirc, B):
    say(f"loss_grad B={B}")
    P = 3000
    pts, lobes, w0 = scene(10, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=4096)
    sm = Samples(pts, lobes, B, 12, 0, 0)
    loss, grad = nirc.nirc_loss_grad(model, dp, sm.queries(nirc), sm.target())
    o_loss, o_grad = sm.loss_grad(pts, w0, W)
    assert abs(float(loss.item()) - o_loss) <= 1e-5 * abs(o_loss)
    assert rel_l2(host(grad), o_grad) <= 1e-5
    # every layer separately
    offs = [0, W * 160, W * 160 + W * W, W * 160 + 2 * W * W, W * 160 + 3 * W * W, o_grad.size]
    for a, b in zip(offs[:-1], offs[1:]):
        assert rel_l2(host(grad)[a:b], o_grad[a:b]) <= 1e-5


@pytest.mark.parametrize("B", [1 << 18, 1 << 20])
def test_loss_grad_large_batches(nirc, B):
    # the training batches of the differentiation workload: activations are recomputed per
    # round inside the gradient kernel (nothing per sample is kept in HBM), partial gradients
    # of at most 256 workgroups are reduced in a fixed order
    say(f"loss_grad large B={B}")
    P = 200_000
    pts, lobes, w0 = scene(31, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=B)
    sm = Samples(pts, lobes, B, 32, 0, 0)
    loss, grad = nirc.nirc_loss_grad(model, dp, sm.queries(nirc), sm.target())
    o_loss, o_grad = sm.loss_grad(pts, w0, W)
    assert abs(float(loss.item()) - o_loss) <= 1e-5 * abs(o_loss)
    assert rel_l2(host(grad), o_grad) <= 1e-5


def test_backward_is_the_loss_vjp(nirc):
    # d_rgb = dloss/dy (frozen denominator) makes the VJP equal the loss gradient
    say("backward")
    P, B = 2000, 777
    pts, lobes, w0 = scene(13, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=B)
    sm = Samples(pts, lobes, B, 14, 0, 0)
    y = oracle.infer(pts, sm.idx, sm.d, w0, W)
    dy = (2.0 * (y - sm.t) / (y * y + 1e-2) / (3.0 * B)).astype(np.float32)
    g = host(nirc.nirc_backward(model, dp, sm.queries(nirc), torch.from_numpy(dy).cuda()))
    # the oracle's VJP with the same FP32 output gradient equals its loss gradient to 1e-7
    _, o_grad = sm.loss_grad(pts, w0, W)
    assert rel_l2(g, o_grad) <= 1e-5


def test_train_step_single_step_parity(nirc):
    say("train_step")
    P, B = 3000, 4096
    pts, lobes, w0 = scene(15, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=B)
    sm = Samples(pts, lobes, B, 16, 0, 0)
    loss = torch.zeros(1, device="cuda")
    nirc.nirc_train_step(model, dp, sm.queries(nirc), sm.target(), loss)
    w1 = host(model.get_weights())
    m, v, step = model.get_adam()
    o_loss, o_grad = sm.loss_grad(pts, w0, W)
    ow = w0.astype(np.float64).copy()
    om = np.zeros_like(ow)
    ov = np.zeros_like(ow)
    oracle.adam(ow, om, ov, o_grad, 1, lr=1e-3)
    assert int(step.item()) == 1
    assert abs(float(loss.item()) - o_loss) <= 1e-5 * o_loss
    assert rel_l2(host(m), om) <= 1e-5
    # first Adam step moves every weight by ~lr * sign(g); compare the update itself
    upd, oupd = w1 - w0, ow - w0
    big = np.abs(o_grad) > 1e-6
    assert np.abs(upd[big] - oupd[big]).max() <= 1e-6
    assert np.abs(upd - oupd).max() <= 1e-3 + 1e-6


def test_train_steps_follow_oracle(nirc):
    # several frames of 4 steps on fresh batches; trajectories compared after every step
    say("train_steps 3 frames")
    P, B = 4096, 4096
    pts, lobes, w0 = scene(17, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=B)
    ow = w0.astype(np.float64).copy()
    om = np.zeros_like(ow)
    ov = np.zeros_like(ow)
    t = 0
    small = np.zeros(ow.shape, bool)   # weights whose oracle gradient was near zero at some step
    for f in range(3):
        for s in range(4):
            sm = Samples(pts, lobes, B, 18, f, s)
            nirc.nirc_train_step(model, dp, sm.queries(nirc), sm.target())
            _, g = sm.loss_grad(pts, ow, W)
            small |= np.abs(g) <= 5e-2 * np.sqrt(np.mean(g * g))
            t += 1
            oracle.adam(ow, om, ov, g, t, lr=1e-3)
    w = host(model.get_weights())
    # FP32 vs FP64 trajectories.  Adam moves a weight by ~lr * sign(g) when |g| is tiny, so a
    # weight whose near-zero gradient changes sign between FP32 and FP64 may differ by up to
    # 2 lr per step; compare the accumulated update in relative L2 and bound all but 0.1 % of
    # the weights to 5 % of the 12-step update scale.
    assert rel_l2(w - w0, ow - w0) <= 1e-2
    assert np.quantile(np.abs(w - ow), 0.999) <= 0.05 * 12 * 1e-3
    # Every weight: no pair of Adam trajectories can drift further apart than twice the largest
    # possible step, lr (1 - b1) / sqrt(1 - b2) = 3.2 lr, in each of the 12 steps.
    assert np.abs(w - ow).max() <= 2 * 12 * 3.17e-3
    # Weights whose gradient stayed above 5 % of its RMS at every step: the FP32 gradient's error
    # is 1e-5 of the vector's norm, i.e. at most 1.5e-3 of the RMS on one of the 22,720 elements,
    # so such a gradient is known to 3 % and Adam's update to ~3 % of lr: the trajectories stay
    # within 12 x 0.03 lr.
    # (Measured: 37 % of the weights qualify, their largest drift 1.5e-5.)
    stable = ~small
    assert stable.mean() > 0.3, stable.mean()
    assert np.abs(w - ow)[stable].max() <= 12 * 0.03 * 1e-3, np.abs(w - ow)[stable].max()


@pytest.mark.parametrize("prec,output", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 2)])
@pytest.mark.parametrize("P,B,steps", [(4096, 4096, 4), (777, 1000, 3), (5000, 65, 1), (3000, 512, 6)])
def test_train_frame_equals_separate_steps(nirc, P, B, steps, prec, output):
    # the one-call frame of training draws the same samples and takes the same Adam steps as
    # tlmc_train_batch + nirc_train_step called step by step (the frame makes the samples of up
    # to 4 steps in one launch; 6 steps take two such launches)
    say("train_frame", P, B, steps, prec, output)
    pts, lobes, w0 = scene(23, P)
    dp = nirc.Points.from_workload(pts)
    cfg = nirc.make_config(precision=prec, output=output)
    a = nirc.Model(w0, cfg=cfg, max_batch=B)
    b = nirc.Model(w0, cfg=cfg, max_batch=B)
    la = torch.zeros(1, device="cuda")
    lb = torch.zeros(1, device="cuda")
    for f in range(2):
        for s in range(steps):
            q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 24, f, s, output)
            nirc.nirc_train_step(a, dp, q, tgt, la)
        nirc.nirc_train_frame(b, dp, lobes, B, steps, 24, f, lb)
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    for x, y in zip(a.get_adam(), b.get_adam()):
        np.testing.assert_array_equal(host(x), host(y))
    assert la.item() == lb.item()
    # a batch larger than the workspace was sized for is refused
    with pytest.raises(nirc.NircError):
        nirc.nirc_train_frame(b, dp, lobes, B + 4096, 1, 24, 0)


def test_nonfinite_gradient_skips_step(nirc):
    say("nonfinite")
    P, B = 500, 256
    pts, lobes, w0 = scene(19, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 20, 0, 0)
    tgt[5, 1] = float("nan")
    nirc.nirc_train_step(model, dp, q, tgt)
    assert model.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD
    np.testing.assert_array_equal(host(model.get_weights()), w0.astype(np.float64))
    _, _, step = model.get_adam()
    assert int(step.item()) == 0
    model.clear_flags()
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 20, 0, 1)
    nirc.nirc_train_step(model, dp, q, tgt)
    assert model.read_flags() == 0
    _, _, step = model.get_adam()
    assert int(step.item()) == 1


def test_determinism(nirc):
    say("determinism")
    P, B = 3000, 3000
    pts, lobes, w0 = scene(21, P)
    dp = nirc.Points.from_workload(pts)
    m1 = nirc.Model(w0, max_batch=B)
    m2 = nirc.Model(w0, max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lobes, B, 22, 0, 0)
    for m in (m1, m2):
        for _ in range(2):
            nirc.nirc_train_step(m, dp, q, tgt)
    np.testing.assert_array_equal(host(m1.get_weights()), host(m2.get_weights()))
    a = host(nirc.tlmc_estimate(m1, dp, lobes, 16, 1, 1))
    b = host(nirc.tlmc_estimate(m2, dp, lobes, 16, 1, 1))
    np.testing.assert_array_equal(a, b)


def test_autograd_function(nirc):
    say("autograd")
    P, Q = 400, 333
    pts, _, w0 = scene(23, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=Q)
    g = torch.Generator().manual_seed(0)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g)
    d = d / d.norm(dim=1, keepdim=True)
    q = nirc.Queries.from_dirs(d.cuda(), idx.cuda())
    w = torch.tensor(w0, device="cuda", requires_grad=True)
    y = nirc.NircFunction.apply(w, model, dp, q)
    up = torch.randn(Q, 3, generator=g).cuda()
    (y * up).sum().backward()
    # finite-difference directional derivative along a random direction, FP64 oracle
    # (small step: a large joint perturbation of all weights flips ReLU masks)
    v = np.random.default_rng(1).normal(size=w0.size)
    h = 1e-6
    yp = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0 + h * v, W)
    ym = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0 - h * v, W)
    fd = ((yp - ym) / (2 * h) * up.cpu().double().numpy()).sum()
    an = float((w.grad.double().cpu().numpy() * v).sum())
    assert an == pytest.approx(fd, rel=1e-4)
    # and the autograd gradient is exactly the library's VJP
    g2 = nirc.nirc_backward(model, dp, q, up)
    np.testing.assert_array_equal(host(w.grad), host(g2))


def test_full_1080p_sampled_points(nirc):
    # the bench configuration: 1920x1080 points, N = 16, checked on sampled points
    say("full-size 1080p N=16 sampled")
    P, N = 1920 * 1080, 16
    pts, lobes, w0 = scene(2, P)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lobes, N, 2, 0, parts=True))
    rng = np.random.default_rng(0)
    sel = np.unique(np.concatenate([rng.choice(P, 3000, replace=False), np.arange(P - 40, P), np.arange(40)]))
    sub = pts.subset(sel)
    # the oracle samples the directions of the selected points by their frame indices
    dirs = oracle.sample_dirs(sub, N, 2, 0, ids=sel)
    o_tl, o_c, o_r = oracle.estimate(sub, lobes, w0, W, N, 2, 0, dirs=dirs)
    check_estimate(tl[sel], c[sel], r[sel], o_tl, o_c, o_r, residual_prediction(sub, w0, W, N, 2, 0, dirs=dirs))
    assert np.isfinite(tl).all()
