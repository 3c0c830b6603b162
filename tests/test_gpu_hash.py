"""The hash-grid cache input (12-level hash grid on x, degree-4 spherical harmonics of w,
identity / one-blob surface values) on the GPU against the FP64 oracle (needs the GPU).

Tolerances are those of the other 16-bit paths: outputs and estimator parts rel-L2 <= 1e-2,
loss and gradients (MLP weights and grid entries) rel-L2 <= ten times the operand format's unit
roundoff.  Grid features are drawn from [-0.5, 0.5] (not the 1e-4 training initialisation) so
that the grid part of every input carries weight in the comparison.  Samples and weights come
from the seeded generator or the oracle, never from the GPU.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import (UNIT_ROUNDOFF, Samples, check_estimate_points, check_query_points, hash_tie_free_samples,
                          host, rel_l2, residual_prediction)

pytestmark = pytest.mark.gpu
PRECS = {"fp32": 0, "bf16": 1, "fp16": 2}
GRAD_TOL = {"fp32": 1e-5, "bf16": 10 * 2.0 ** -9, "fp16": 10 * 2.0 ** -12}
GRIDS = {"default": (18, 16, 1.5), "small": (10, 4, 1.5)}
# 10,069 entries: an odd count, so the parameter vector's length is 2 mod 4 and the 4-wide Adam
# and gradient-scaling passes run their ragged tails
ODD_GRID = (10, 4, 1.4)


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def _model(nirc, prec, grid, seed, max_batch=0, scale=0.5, **cfg):
    w = wl.make_hash_weights(seed, 64, 2 * oracle.hash_entries(grid), scale)
    g = nirc.make_hash_grid(*grid)
    m = nirc.HashModel(w, cfg=nirc.make_config(precision=PRECS[prec], **cfg), grid=g, max_batch=max_batch)
    return m, w


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("grid", ["default", "small"])
@pytest.mark.parametrize("Q", [1, 1000, 4099])
def test_hash_infer(nirc, prec, grid, Q):
    print(f"hash infer {prec} {grid} Q={Q}", flush=True)
    P = 700
    pts = wl.make_points(41, P)
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, prec, GRIDS[grid], 41)
    g = torch.Generator().manual_seed(Q)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g)
    d = d / d.norm(dim=1, keepdim=True)
    y = host(nirc.nirc_hash_infer(model, dp, nirc.Queries.from_dirs(d.cuda(), idx.cuda())))
    ref = oracle.hash_infer(pts, idx.numpy(), d.double().numpy(), w, 64, GRIDS[grid])
    e = rel_l2(y, ref)
    print(f"  rel-L2 {e:.3e}", flush=True)
    assert e <= 1e-2
    check_query_points(f"hash infer {prec}", y, ref, prec)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("P,N", [(17, 3), (4096, 8), (1000, 16), (100, 64), (4001, 5)])
def test_hash_estimate(nirc, prec, P, N):
    print(f"hash estimate {prec} P={P} N={N}", flush=True)
    pts = wl.make_points(42, P)
    lob = wl.make_lobes(42).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, prec, GRIDS["default"], 42)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, lob, N, 9, 1, parts=True))
    o_tl, o_c, o_r = oracle.hash_estimate(pts, lob, w, N, 9, 1)
    print(f"  F_c rel-L2 {rel_l2(c, o_c):.3e}  F_tl {rel_l2(tl, o_tl):.3e}", flush=True)
    assert rel_l2(c, o_c) <= 1e-2
    assert rel_l2(tl, o_tl) <= 1e-2
    assert np.linalg.norm(r - o_r) <= 1e-2 * np.linalg.norm(o_c)
    check_estimate_points(f"hash estimate {prec}", tl, c, r, o_tl, o_c, o_r,
                          residual_prediction(pts, w, 64, N, 9, 1, hash_grid=GRIDS["default"]), prec)


def test_hash_estimate_caller_residual(nirc):
    P, N = 999, 16
    pts = wl.make_points(43, P)
    lob = wl.make_lobes(43).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, "bf16", GRIDS["default"], 43)
    rr = np.random.default_rng(43).random((P, 3)).astype(np.float32)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, None, N, 4, 2, parts=True,
                                                         residual=torch.from_numpy(rr).cuda()))
    o_tl, o_c, o_r = oracle.hash_estimate(pts, lob, w, N, 4, 2, rrad=rr.astype(np.float64))
    assert rel_l2(c, o_c) <= 1e-2
    assert np.linalg.norm(r - o_r) <= 1e-2 * np.linalg.norm(o_c)


def test_hash_full_1080p_sampled_points(nirc):
    # the full frame (1920 x 1080 points, N = 16, BF16) checked on sampled points, ragged tail
    # included (the oracle samples their directions by frame index)
    print("hash 1080p N=16 sampled", flush=True)
    P, N = 1920 * 1080, 16
    pts = wl.make_points(44, P)
    lob = wl.make_lobes(44).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, "bf16", GRIDS["default"], 44)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, lob, N, 3, 1, parts=True))
    rng = np.random.default_rng(2)
    sel = np.unique(np.concatenate([rng.choice(P, 2000, replace=False), np.arange(P - 23, P)]))
    sub = pts.subset(sel)
    dirs = oracle.sample_dirs(sub, N, 3, 1, ids=sel)
    o_tl, o_c, o_r = oracle.hash_estimate(sub, lob, w, N, 3, 1, dirs=dirs)
    assert rel_l2(c[sel], o_c) <= 1e-2
    assert np.linalg.norm(tl[sel] - o_tl) <= 1e-2 * np.linalg.norm(o_c)
    check_estimate_points("hash 1080p sampled", tl[sel], c[sel], r[sel], o_tl, o_c, o_r,
                          residual_prediction(sub, w, 64, N, 3, 1, dirs=dirs, hash_grid=GRIDS["default"]), "bf16")
    assert np.isfinite(tl).all()


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("grid", ["default", "small"])
@pytest.mark.parametrize("B,kind", [(1, 0), (1000, 0), (65536, 0), (4096, 1)])
def test_hash_loss_grad(nirc, prec, grid, B, kind):
    print(f"hash loss_grad {prec} {grid} B={B} kind={kind}", flush=True)
    P = 3000
    pts = wl.make_points(45, P)
    lob = wl.make_lobes(45).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, prec, GRIDS[grid], 45, max_batch=B, loss=kind)
    sm = Samples(pts, lob, B, 46, 0, 0)
    loss, grad = nirc.nirc_hash_loss_grad(model, dp, sm.queries(nirc), sm.target())
    w64 = w.astype(np.float64)
    o_loss, o_grad = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w64, 64, GRIDS[grid], kind=kind)
    g = host(grad)
    nm = oracle.hash_mlp_params(64)
    e_loss = abs(float(loss.item()) - o_loss) / abs(o_loss)
    e_mlp = rel_l2(g[:nm], o_grad[:nm])
    assert e_loss <= GRAD_TOL[prec]
    assert e_mlp <= GRAD_TOL[prec]
    # A grid entry's gradient sums over a handful of samples, so one hidden unit that 16-bit
    # rounding switches the other way (a pre-activation within rounding of zero) moves it by a
    # large fraction, where the MLP gradients average such switches away.  The grid part is
    # therefore compared, against the same plain FP64 oracle, on samples none of whose units lies
    # within 8 sigma of its switch (relu_tie_mask: sigma is the spread operand rounding gives the
    # pre-activation); on them both sides take every ReLU decision alike.
    tf, frac = hash_tie_free_samples(pts, lob, B, 46, 0, 0, w64, GRIDS[grid], UNIT_ROUNDOFF[prec])
    _, gt = nirc.nirc_hash_loss_grad(model, dp, tf.queries(nirc), tf.target())
    _, ot = oracle.hash_loss_grad(pts, tf.idx, tf.d, tf.t, w64, 64, GRIDS[grid], kind=kind)
    gt = host(gt)
    e_tab = rel_l2(gt[nm:], ot[nm:])
    print(f"  loss {e_loss:.3e}  mlp {e_mlp:.3e}  grid {e_tab:.3e} on {tf.idx.size} tie-free samples "
          f"({100 * frac:.1f}% of candidates; all {B} samples: grid {rel_l2(g[nm:], o_grad[nm:]):.3e})", flush=True)
    assert tf.idx.size == B or tf.idx.size >= 4096
    assert e_tab <= GRAD_TOL[prec]
    assert rel_l2(gt[:nm], ot[:nm]) <= GRAD_TOL[prec]
    res, off, _ = oracle.hash_levels(GRIDS[grid])
    ends = list(off[1:]) + [oracle.hash_entries(GRIDS[grid])]
    for l in range(12):
        a, b = 2 * off[l], 2 * ends[l]
        tl_ = w64[nm + a:nm + b]
        got_l = float(np.dot(tl_, gt[nm + a:nm + b]))
        ref_l = float(np.dot(tl_, ot[nm + a:nm + b]))
        assert abs(got_l - ref_l) <= GRAD_TOL[prec] * float(np.abs(tl_ * ot[nm + a:nm + b]).sum()) + 1e-30, l
    # entries no sample touches stay exactly zero
    assert np.all(g[nm:][o_grad[nm:] == 0.0] == 0.0)
    assert np.all(gt[nm:][ot[nm:] == 0.0] == 0.0)
    # <table, grid gradient> = <W1 grid columns, their gradient> (both are sum_b sum_k e_bk de_bk)
    W1 = w64[:64 * 64].reshape(64, 64)[:, :24]
    lhs = float(np.dot(w64[nm:], g[nm:]))
    rhs = float(np.sum(W1 * g[:64 * 64].reshape(64, 64)[:, :24]))
    assert abs(lhs - rhs) <= GRAD_TOL[prec] * float(np.abs(W1 * g[:64 * 64].reshape(64, 64)[:, :24]).sum())


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("grid", [GRIDS["small"], ODD_GRID])
def test_hash_adam_step_matches_oracle(nirc, prec, grid):
    # one Adam step from zero moments with the oracle's gradient given to both sides
    P, B = 2000, 4096
    pts = wl.make_points(47, P)
    lob = wl.make_lobes(47).packed()
    model, w = _model(nirc, prec, grid, 47, max_batch=B)
    assert model.n_params % 4 == (2 if grid == ODD_GRID else 0)
    sm = Samples(pts, lob, B, 48, 0, 0)
    _, g = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w.astype(np.float64), 64, grid)
    g32 = g.astype(np.float32)
    g32[-3:] = [3e-3, -2e-3, 1e-3]   # the last entries (a 4-wide pass's tail) take a step as well
    nirc.nirc_hash_adam_step(model, torch.from_numpy(g32).cuda())
    got = host(model.get_weights())
    wo = w.astype(np.float64)
    m = np.zeros_like(wo)
    v = np.zeros_like(wo)
    w_start = w.astype(np.float64)
    oracle.adam(wo, m, v, g32.astype(np.float64), 1)
    np.testing.assert_allclose(got, wo, rtol=0, atol=2e-6)
    assert np.all(np.abs(got[-3:] - w_start[-3:]) > 5e-4)
    assert model.read_flags() == 0


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("grid", [GRIDS["small"], ODD_GRID])
def test_hash_nonfinite_gradient_skips_step(nirc, prec, grid):
    model, w = _model(nirc, prec, grid, 49, max_batch=16)
    g = np.zeros(model.n_params, np.float32)
    g[-1] = np.nan
    nirc.nirc_hash_adam_step(model, torch.from_numpy(g).cuda())
    np.testing.assert_array_equal(host(model.get_weights()), w.astype(np.float64))
    assert model.read_flags() & nirc.NIRC_FLAG_NONFINITE_GRAD


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hash_training_reduces_cache_error(nirc, prec):
    # online training from the 1e-4 grid initialisation: the cache's relative L2 error on held-out
    # samples falls well below its start within 30 frames of 4 steps
    print(f"hash training {prec}", flush=True)
    P, B = 65536, 16384
    pts = wl.make_points(50, P)
    lob = wl.make_lobes(50).packed()
    dp = nirc.Points.from_workload(pts)
    model, _ = _model(nirc, prec, GRIDS["default"], 50, max_batch=B, scale=1e-4)
    held = Samples(pts, lob, 8192, 51, 999, 0)
    q = held.queries(nirc)

    def err():
        return rel_l2(host(nirc.nirc_hash_infer(model, dp, q)), held.t)

    e0 = err()
    for f in range(30):
        for s in range(4):
            qq, tgt = nirc.tlmc_train_batch(dp, lob, B, 52, f, s)
            nirc.nirc_hash_train_step(model, dp, qq, tgt)
    e1 = err()
    print(f"  cache rel-L2 {e0:.3f} -> {e1:.3f}", flush=True)
    assert model.read_flags() == 0
    assert e1 < 0.35 * e0 and e1 < 0.3


def test_hash_estimator_unbiased_over_seeds(nirc):
    # E[F_tl] = F whatever the cache: mean over seeds against the closed-form integral
    P, N, S = 64, 4, 400
    pts = wl.make_points(53, P)
    lob = wl.make_lobes(53).packed()
    dp = nirc.Points.from_workload(pts)
    model, _ = _model(nirc, "bf16", GRIDS["default"], 53)
    F = oracle.closed_form(pts, lob)
    samples = np.stack([host(nirc.nirc_hash_estimate(model, dp, lob, N, 3000 + s, 0)) for s in range(S)])
    z = (samples.mean(axis=0) - F) / (samples.std(axis=0, ddof=1) / math.sqrt(S))
    assert np.abs(z).max() < 5.0


def test_hash_rejects_unsupported_configurations(nirc):
    w = wl.make_hash_weights(1, 64, 2 * oracle.hash_entries(GRIDS["small"]))
    g = nirc.make_hash_grid(*GRIDS["small"])
    for cfg in (nirc.make_config(width=128, precision=1),
                nirc.make_config(precision=1, loss=2), nirc.make_config(precision=1, output=1)):
        with pytest.raises(nirc.NircError):
            nirc.HashModel(w, cfg=cfg, grid=g, max_batch=0)
    with pytest.raises(nirc.NircError):
        nirc.HashModel(w, cfg=nirc.make_config(precision=1), grid=nirc.make_hash_grid(9, 16, 1.5), max_batch=0)


@pytest.mark.parametrize("P,N", [(3, 1), (5, 4096), (33, 2), (16, 9)])
def test_hash_estimate_edge_counts(nirc, P, N):
    # smallest and largest direction counts, a group smaller than a tile, N not dividing 16
    print(f"hash edge P={P} N={N}", flush=True)
    pts = wl.make_points(54, P)
    lob = wl.make_lobes(54).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, "bf16", GRIDS["small"], 54)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, lob, N, 2, 0, parts=True))
    o_tl, o_c, o_r = oracle.hash_estimate(pts, lob, w, N, 2, 0, grid=GRIDS["small"])
    assert rel_l2(c, o_c) <= 1e-2
    assert np.linalg.norm(r - o_r) <= 1e-2 * np.linalg.norm(o_c)
    check_estimate_points(f"hash edge P={P} N={N}", tl, c, r, o_tl, o_c, o_r,
                          residual_prediction(pts, w, 64, N, 2, 0, hash_grid=GRIDS["small"]), "bf16")


def test_hash_empty_inputs(nirc):
    model, _ = _model(nirc, "bf16", GRIDS["small"], 55)
    empty = nirc.Points.from_workload(wl.make_points(55, 0))
    lob = wl.make_lobes(55).packed()
    assert nirc.nirc_hash_estimate(model, empty, lob, 8, 0, 0).shape == (0, 3)
    q = nirc.Queries.from_dirs(torch.zeros((0, 3), device="cuda"))
    assert nirc.nirc_hash_infer(model, empty, q).shape == (0, 3)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hash_checkpoint_resume(nirc, prec):
    # a restored checkpoint is the saved state bit for bit (and answers identically); training on
    # from it follows the original bit for bit (the grid gradient is summed in fixed point, so
    # the order of its atomic adds does not matter)
    P, B = 4096, 4096
    pts = wl.make_points(56, P)
    lob = wl.make_lobes(56).packed()
    dp = nirc.Points.from_workload(pts)
    a, _ = _model(nirc, prec, GRIDS["small"], 56, max_batch=B, scale=1e-4)
    b, _ = _model(nirc, prec, GRIDS["small"], 57, max_batch=B, scale=1e-4)

    def frames(m, f0):
        for f in range(f0, f0 + 2):
            for s_ in range(2):
                q, tgt = nirc.tlmc_train_batch(dp, lob, B, 58, f, s_)
                nirc.nirc_hash_train_step(m, dp, q, tgt)

    frames(a, 0)
    blob = a.get_state()
    wc = host(a.get_weights())
    q = nirc.Queries.from_dirs(torch.nn.functional.normalize(torch.randn(100, 3, device="cuda"), dim=1))
    ya = host(nirc.nirc_hash_infer(a, dp, q))
    b.set_state(blob)
    np.testing.assert_array_equal(host(b.get_state()), host(blob))
    np.testing.assert_array_equal(host(nirc.nirc_hash_infer(b, dp, q)), ya)
    frames(a, 2)
    frames(b, 2)
    # (the blobs' alignment padding is not state: compare what the updates produce)
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    assert a.read_flags() == 0 and b.read_flags() == 0


@pytest.mark.parametrize("prec", ["fp32", "fp16"])
def test_hash_positions_outside_the_unit_cube(nirc, prec):
    # positions are clamped to the grid's domain on both sides: points scattered over [-0.25, 1.25]^3,
    # in the estimate and in the gradient (whose scatter then lands on the cube's faces)
    P, N, B = 1000, 8, 4096
    pts = wl.make_points(59, P)
    for a in (pts.px, pts.py, pts.pz):
        a[:] = (a * 1.5 - 0.25).astype(np.float32)
    lob = wl.make_lobes(59).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, prec, GRIDS["default"], 59, max_batch=B)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, lob, N, 5, 0, parts=True))
    o_tl, o_c, o_r = oracle.hash_estimate(pts, lob, w, N, 5, 0)
    assert rel_l2(c, o_c) <= (HASH_F32_TOL if prec == "fp32" else 1e-2)
    assert np.isfinite(tl).all()
    w64 = w.astype(np.float64)
    # tie-free samples (as in test_hash_loss_grad), so that the grid part is held to the bound
    sm, _ = hash_tie_free_samples(pts, lob, B, 69, 0, 0, w64, GRIDS["default"], UNIT_ROUNDOFF[prec])
    _, grad = nirc.nirc_hash_loss_grad(model, dp, sm.queries(nirc), sm.target())
    g = host(grad)
    _, o_grad = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w64, 64, GRIDS["default"])
    nm = oracle.hash_mlp_params(64)
    e_mlp, e_tab = rel_l2(g[:nm], o_grad[:nm]), rel_l2(g[nm:], o_grad[nm:])
    print(f"hash outside the cube {prec}: F_c {rel_l2(c, o_c):.3e} mlp {e_mlp:.3e} grid {e_tab:.3e}", flush=True)
    assert e_mlp <= GRAD_TOL[prec]
    assert e_tab <= (HASH_F32_GRID_TOL if prec == "fp32" else GRAD_TOL[prec])
    assert np.all(g[nm:][o_grad[nm:] == 0.0] == 0.0)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hash_train_frame_matches_step_loop(nirc, prec):
    # the native frame loop (samples generated into the workspace) against the same steps called
    # one by one: bit for bit
    P, B = 4096, 2048
    pts = wl.make_points(60, P)
    lob = wl.make_lobes(60).packed()
    dp = nirc.Points.from_workload(pts)
    a, w = _model(nirc, prec, GRIDS["small"], 60, max_batch=B, scale=1e-4)
    b, _ = _model(nirc, prec, GRIDS["small"], 60, max_batch=B, scale=1e-4)
    loss = torch.zeros(1, device="cuda")
    for f in range(2):
        nirc.nirc_hash_train_frame(a, dp, lob, B, 3, 61, f, loss)
        for s_ in range(3):
            q, tgt = nirc.tlmc_train_batch(dp, lob, B, 61, f, s_)
            nirc.nirc_hash_train_step(b, dp, q, tgt)
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    assert np.isfinite(float(loss.item())) and float(loss.item()) > 0


# FP32 hash-grid model: the FP32 bound of the frequency model, 1e-5 (measured: outputs ~4e-8, F_c <= 2e-7, F_tl <= 3e-7 of |F_c|; a
# position whose FP32 product with N_l rounds across a cell edge moves its grid value by at most
# 2^-24 N_l of a cell times a corner difference, rare and continuous).
HASH_F32_TOL = 1e-5


@pytest.mark.parametrize("grid", ["default", "small"])
@pytest.mark.parametrize("Q", [1, 1000, 4099])
def test_hash_infer_fp32(nirc, grid, Q):
    P = 700
    pts = wl.make_points(62, P)
    dp = nirc.Points.from_workload(pts)
    w = wl.make_hash_weights(62, 64, 2 * oracle.hash_entries(GRIDS[grid]), 0.5)
    model = nirc.HashModel(w, cfg=nirc.make_config(precision=0), grid=nirc.make_hash_grid(*GRIDS[grid]), max_batch=0)
    g = torch.Generator().manual_seed(Q)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g)
    d = d / d.norm(dim=1, keepdim=True)
    y = host(nirc.nirc_hash_infer(model, dp, nirc.Queries.from_dirs(d.cuda(), idx.cuda())))
    ref = oracle.hash_infer(pts, idx.numpy(), d.double().numpy(), w, 64, GRIDS[grid])
    e = rel_l2(y, ref)
    print(f"hash infer fp32 {grid} Q={Q}: rel-L2 {e:.3e}", flush=True)
    assert e <= HASH_F32_TOL
    check_query_points("hash infer fp32", y, ref, "fp32")


@pytest.mark.parametrize("P,N", [(17, 3), (4096, 8), (1000, 16), (100, 64), (4001, 5)])
def test_hash_estimate_fp32(nirc, P, N):
    pts = wl.make_points(63, P)
    lob = wl.make_lobes(63).packed()
    dp = nirc.Points.from_workload(pts)
    w = wl.make_hash_weights(63, 64, 2 * oracle.hash_entries(GRIDS["default"]), 0.5)
    model = nirc.HashModel(w, cfg=nirc.make_config(precision=0), grid=nirc.make_hash_grid(*GRIDS["default"]),
                           max_batch=0)
    tl, c, r = (host(t) for t in nirc.nirc_hash_estimate(model, dp, lob, N, 9, 1, parts=True))
    o_tl, o_c, o_r = oracle.hash_estimate(pts, lob, w, N, 9, 1)
    print(f"hash estimate fp32 P={P} N={N}: F_c {rel_l2(c, o_c):.3e} F_tl {np.linalg.norm(tl - o_tl) / np.linalg.norm(o_c):.3e}",
          flush=True)
    assert rel_l2(c, o_c) <= HASH_F32_TOL
    assert np.linalg.norm(tl - o_tl) <= HASH_F32_TOL * np.linalg.norm(o_c)
    assert np.linalg.norm(r - o_r) <= HASH_F32_TOL * np.linalg.norm(o_c)
    check_estimate_points("hash estimate fp32", tl, c, r, o_tl, o_c, o_r,
                          residual_prediction(pts, w, 64, N, 9, 1, hash_grid=GRIDS["default"]), "fp32")


# FP32 grid-entry gradients entry by entry.  In FP32 a ReLU decision flips only for a unit within
# FP32 rounding of zero (about one in 10^6 decisions, so a few samples in 65,536), but such a
# sample's entries then lose or gain one unit's whole contribution, which a grid entry's sum over
# few samples does not average away.  The per-level sums (weighted by the table) do average it, but
# at B = 65,536 on the 2^10-entry table a level's weighted sum cancels to a small fraction of its
# absolute sum, so they are held to ten times the MLP bound (measured: 1.2e-5 at worst).
HASH_F32_GRID_TOL = 1e-3
HASH_F32_LEVEL_TOL = 1e-4


@pytest.mark.parametrize("grid", ["default", "small"])
@pytest.mark.parametrize("B,kind", [(1, 0), (1000, 0), (65536, 0), (4096, 1)])
def test_hash_loss_grad_fp32(nirc, grid, B, kind):
    print(f"hash loss_grad fp32 {grid} B={B} kind={kind}", flush=True)
    P = 3000
    pts = wl.make_points(45, P)
    lob = wl.make_lobes(45).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, "fp32", GRIDS[grid], 45, max_batch=B, loss=kind)
    sm = Samples(pts, lob, B, 46, 0, 0)
    loss, grad = nirc.nirc_hash_loss_grad(model, dp, sm.queries(nirc), sm.target())
    w64 = w.astype(np.float64)
    o_loss, o_grad = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w64, 64, GRIDS[grid], kind=kind)
    g = host(grad)
    nm = oracle.hash_mlp_params(64)
    e_loss = abs(float(loss.item()) - o_loss) / abs(o_loss)
    e_mlp = rel_l2(g[:nm], o_grad[:nm])
    e_tab = rel_l2(g[nm:], o_grad[nm:])
    print(f"  loss {e_loss:.3e}  mlp {e_mlp:.3e}  grid {e_tab:.3e}", flush=True)
    assert e_loss <= GRAD_TOL["fp32"]
    assert e_mlp <= GRAD_TOL["fp32"]
    assert e_tab <= HASH_F32_GRID_TOL
    res, off, _ = oracle.hash_levels(GRIDS[grid])
    ends = list(off[1:]) + [oracle.hash_entries(GRIDS[grid])]
    for l in range(12):
        a, b = 2 * off[l], 2 * ends[l]
        tl_ = w64[nm + a:nm + b]
        got_l = float(np.dot(tl_, g[nm + a:nm + b]))
        ref_l = float(np.dot(tl_, o_grad[nm + a:nm + b]))
        assert abs(got_l - ref_l) <= HASH_F32_LEVEL_TOL * float(np.abs(tl_ * o_grad[nm + a:nm + b]).sum()) + 1e-30, l
    assert np.all(g[nm:][o_grad[nm:] == 0.0] == 0.0)
    W1 = w64[:64 * 64].reshape(64, 64)[:, :24]
    lhs = float(np.dot(w64[nm:], g[nm:]))
    rhs = float(np.sum(W1 * g[:64 * 64].reshape(64, 64)[:, :24]))
    assert abs(lhs - rhs) <= GRAD_TOL["fp32"] * float(np.abs(W1 * g[:64 * 64].reshape(64, 64)[:, :24]).sum())
    # on samples with no unit within FP32 rounding of its switch (relu_tie_mask with sixteen
    # times FP32's unit roundoff, for the accumulation order) the grid entries meet the MLP bound
    tf, _ = hash_tie_free_samples(pts, lob, B, 46, 0, 0, w64, GRIDS[grid], 16 * UNIT_ROUNDOFF["fp32"])
    _, gt = nirc.nirc_hash_loss_grad(model, dp, tf.queries(nirc), tf.target())
    _, ot = oracle.hash_loss_grad(pts, tf.idx, tf.d, tf.t, w64, 64, GRIDS[grid], kind=kind)
    e_tf = rel_l2(host(gt)[nm:], ot[nm:])
    print(f"  grid on {tf.idx.size} tie-free samples {e_tf:.3e}", flush=True)
    assert e_tf <= GRAD_TOL["fp32"]


def test_hash_fp32_train_steps_refresh_the_packed_layers(nirc):
    # after FP32 training steps the FP32 inference reads the updated parameters: its outputs match
    # the oracle evaluated on the parameters the model reports, and every step was committed
    P, B = 3000, 4096
    pts = wl.make_points(66, P)
    lob = wl.make_lobes(66).packed()
    dp = nirc.Points.from_workload(pts)
    model, w = _model(nirc, "fp32", GRIDS["small"], 66, max_batch=B)
    for s_ in range(3):
        q, tgt = nirc.tlmc_train_batch(dp, lob, B, 67, 0, s_)
        nirc.nirc_hash_train_step(model, dp, q, tgt)
    assert model.read_flags() == 0
    w1 = host(model.get_weights())
    assert rel_l2(w1, w.astype(np.float64)) > 1e-4
    sm = Samples(pts, lob, 2000, 68, 0, 0)
    y = host(nirc.nirc_hash_infer(model, dp, sm.queries(nirc)))
    ref = oracle.hash_infer(pts, sm.idx, sm.d, w1.astype(np.float32), 64, GRIDS["small"])
    e = rel_l2(y, ref)
    print(f"hash fp32 after 3 steps: infer rel-L2 {e:.3e}", flush=True)
    assert e <= HASH_F32_TOL


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
def test_hash_grid_gradient_without_relu_decisions(nirc, prec):
    # a network whose every pre-activation is positive (non-negative grid features and first-layer
    # grid columns, a positive albedo bias, positive hidden weights, no direction or other surface
    # columns) takes no ReLU decision that rounding could flip, so the grid-entry gradient (the
    # TS product and the scatter) is held to the rounding bound entry by entry
    print(f"hash grid gradient, positive network, {prec}", flush=True)
    grid = GRIDS["default"]
    rng = np.random.default_rng(70)
    n_tab = 2 * oracle.hash_entries(grid)
    W1 = np.zeros((64, 64))
    W1[:, :24] = rng.uniform(0.0, 2.0 / 24, (64, 24))
    W1[:, 60:63] = rng.uniform(0.1, 0.3, (64, 3))
    hid = [rng.uniform(0.0, 2.0 / 64, (64, 64)) for _ in range(3)]
    W5 = rng.uniform(-0.05, 0.05, (3, 64))
    table = rng.uniform(0.0, 0.5, n_tab)
    w = np.concatenate([W1.ravel()] + [h.ravel() for h in hid] + [W5.ravel(), table]).astype(np.float32)
    P, B = 3000, 16384
    pts = wl.make_points(71, P)
    lob = wl.make_lobes(71).packed()
    dp = nirc.Points.from_workload(pts)
    model = nirc.HashModel(w, cfg=nirc.make_config(precision=PRECS[prec]), grid=nirc.make_hash_grid(*grid),
                           max_batch=B)
    sm = Samples(pts, lob, B, 72, 0, 0)
    loss, grad = nirc.nirc_hash_loss_grad(model, dp, sm.queries(nirc), sm.target())
    o_loss, o_grad = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w.astype(np.float64), 64, grid)
    g = host(grad)
    nm = oracle.hash_mlp_params(64)
    e_mlp = rel_l2(g[:nm], o_grad[:nm])
    e_tab = rel_l2(g[nm:], o_grad[nm:])
    print(f"  mlp {e_mlp:.3e}  grid {e_tab:.3e}", flush=True)
    assert e_mlp <= GRAD_TOL[prec]
    assert e_tab <= GRAD_TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_hash_gradient_is_deterministic(nirc, prec):
    # the same batch twice (and on a second model): identical gradients, bit for bit, although
    # the grid part is gathered by atomic adds from every workgroup
    P, B = 3000, 65536
    pts = wl.make_points(62, P)
    lob = wl.make_lobes(62).packed()
    dp = nirc.Points.from_workload(pts)
    m1, _ = _model(nirc, prec, GRIDS["default"], 62, max_batch=B)
    m2, _ = _model(nirc, prec, GRIDS["default"], 62, max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lob, B, 63, 0, 0)
    g = [host(nirc.nirc_hash_loss_grad(m, dp, q, tgt)[1]) for m in (m1, m1, m2)]
    np.testing.assert_array_equal(g[0], g[1])
    np.testing.assert_array_equal(g[0], g[2])
    assert np.count_nonzero(g[0][oracle.hash_mlp_params(64):]) > 1000
