"""BF16 / FP16 MFMA paths against the FP64 oracle (needs the GPU).

Tolerances: cache outputs and estimator outputs rel-L2 <= 1e-2 (16-bit operands, FP32
accumulation; the estimator against the oracle's own directions); estimator MRSE within 2 % of
the FP32 path on identical weights, seeds and directions.  Training samples are drawn by the
oracle and given to both sides.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import Samples, check_estimate_points, check_query_points, host, rel_l2, residual_prediction

pytestmark = pytest.mark.gpu
W = 64
PRECS = {"bf16": 1, "fp16": 2}
# gradient tolerance: ten times the unit roundoff of the operand format (BF16 2^-9, FP16
# 2^-12), for roundings that compound through four forward and four backward layers
GRAD_TOL = {"bf16": 10 * 2.0 ** -9, "fp16": 10 * 2.0 ** -12}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("Q", [1, 1000, 4099])
def test_infer_16bit(nirc, prec, Q):
    print(f"infer {prec} Q={Q}", flush=True)
    P = 500
    pts = wl.make_points(31, P)
    w0 = wl.make_weights(31, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=0)
    g = torch.Generator().manual_seed(Q)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g)
    d = d / d.norm(dim=1, keepdim=True)
    y = host(nirc.nirc_infer(model, dp, nirc.Queries.from_dirs(d.cuda(), idx.cuda())))
    ref = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0, W)
    assert rel_l2(y, ref) <= 1e-2
    check_query_points(f"infer {prec} Q={Q}", y, ref, prec)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("P,N", [(17, 3), (4096, 8), (1000, 16), (100, 64), (4001, 5), (1003, 1), (333, 24)])
def test_estimate_16bit(nirc, prec, P, N):
    print(f"estimate {prec} P={P} N={N}", flush=True)
    pts = wl.make_points(32, P)
    lob = wl.make_lobes(32).packed()
    w0 = wl.make_weights(32, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lob, N, 9, 1, parts=True))
    o_tl, o_c, o_r = oracle.estimate(pts, lob, w0, W, N, 9, 1)
    assert rel_l2(c, o_c) <= 1e-2
    assert rel_l2(tl, o_tl) <= 1e-2
    assert np.linalg.norm(r - o_r) <= 1e-2 * np.linalg.norm(o_c)
    check_estimate_points(f"estimate {prec} P={P} N={N}", tl, c, r, o_tl, o_c, o_r,
                          residual_prediction(pts, w0, W, N, 9, 1), prec)


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
@pytest.mark.parametrize("B", [1, 1000, 65536])
def test_loss_grad_16bit(nirc, prec, B):
    # 16-bit forward and backward operands (FP32 accumulation, FP32 output gradient) against the
    # FP64 gradient on the same samples
    print(f"loss_grad {prec} B={B}", flush=True)
    P = 3000
    pts = wl.make_points(35, P)
    lob = wl.make_lobes(35).packed()
    w0 = wl.make_weights(35, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=B)
    sm = Samples(pts, lob, B, 36, 0, 0)
    loss, grad = nirc.nirc_loss_grad(model, dp, sm.queries(nirc), sm.target())
    o_loss, o_grad = sm.loss_grad(pts, w0, W)
    e_loss = abs(float(loss.item()) - o_loss) / abs(o_loss)
    e_grad = rel_l2(host(grad), o_grad)
    print(f"  loss rel err {e_loss:.3e}  grad rel-L2 {e_grad:.3e}", flush=True)
    assert e_loss <= GRAD_TOL[prec]
    assert e_grad <= GRAD_TOL[prec]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_mrse_within_two_percent_of_fp32(nirc, prec):
    print(f"mrse {prec}", flush=True)
    P, N = 65536, 16
    pts = wl.make_points(33, P)
    lob = wl.make_lobes(33).packed()
    w0 = wl.make_weights(33, W)
    dp = nirc.Points.from_workload(pts)
    table = nirc.tlmc_reference_table(lob)
    out = {}
    for name, pr in (("fp32", 0), (prec, PRECS[prec])):
        model = nirc.Model(w0, cfg=nirc.make_config(precision=pr), max_batch=65536)
        # train a few frames so that the cache is not random, identically for both precisions
        for f in range(3):
            for s in range(4):
                q, tgt = nirc.tlmc_train_batch(dp, lob, 65536, 5, f, s)
                nirc.nirc_train_step(model, dp, q, tgt)
        tl = nirc.tlmc_estimate(model, dp, lob, N, 5, 3)
        out[name] = float(nirc.tlmc_frame_stats(dp, lob, table, tl)[4].item())
    print(out, flush=True)
    assert abs(out[prec] - out["fp32"]) <= 0.02 * out["fp32"]


@pytest.mark.parametrize("prec", ["bf16", "fp16"])
def test_train_step_refreshes_16bit_copy(nirc, prec):
    # training keeps FP32 master weights; after a step the 16-bit copy the kernels read must
    # follow the new master weights: the trained model answers exactly as a model built from
    # its master weights, and within 16-bit tolerance of the FP32 model on the same weights
    print(f"train refresh {prec}", flush=True)
    P, B = 3000, 4096
    pts = wl.make_points(34, P)
    lob = wl.make_lobes(34).packed()
    w0 = wl.make_weights(34, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=B)
    for s in range(3):
        q, tgt = nirc.tlmc_train_batch(dp, lob, B, 7, 0, s)
        nirc.nirc_train_step(model, dp, q, tgt)
    w = model.get_weights()
    assert np.abs(host(w) - w0).max() > 1e-3
    fresh = nirc.Model(w, cfg=nirc.make_config(precision=PRECS[prec]), max_batch=0)
    f32 = nirc.Model(w, max_batch=0)
    sm = Samples(pts, lob, 5000, 8, 0, 0)
    q = sm.queries(nirc)
    y = host(nirc.nirc_infer(model, dp, q))
    np.testing.assert_array_equal(y, host(nirc.nirc_infer(fresh, dp, q)))
    assert rel_l2(y, host(nirc.nirc_infer(f32, dp, q))) <= 1e-2
    np.testing.assert_array_equal(host(nirc.tlmc_estimate(model, dp, lob, 8, 1, 0)),
                                  host(nirc.tlmc_estimate(fresh, dp, lob, 8, 1, 0)))


def test_full_4k_bf16_sampled_points(nirc):
    # the largest serving frame: 3840 x 2160 points, N = 32, BF16, checked on sampled points
    # (the oracle samples their directions by frame index) including the ragged tail
    print("4K N=32 BF16 sampled", flush=True)
    P, N = 3840 * 2160, 32
    pts = wl.make_points(37, P)
    lob = wl.make_lobes(37).packed()
    w0 = wl.make_weights(37, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS["bf16"]), max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lob, N, 3, 1, parts=True))
    rng = np.random.default_rng(1)
    sel = np.unique(np.concatenate([rng.choice(P, 2000, replace=False), np.arange(P - 23, P)]))
    sub = pts.subset(sel)
    dirs = oracle.sample_dirs(sub, N, 3, 1, ids=sel)
    o_tl, o_c, o_r = oracle.estimate(sub, lob, w0, W, N, 3, 1, dirs=dirs)
    assert rel_l2(c[sel], o_c) <= 1e-2
    assert np.linalg.norm(tl[sel] - o_tl) <= 1e-2 * np.linalg.norm(o_c)
    check_estimate_points("4K sampled", tl[sel], c[sel], r[sel], o_tl, o_c, o_r,
                          residual_prediction(sub, w0, W, N, 3, 1, dirs=dirs), "bf16")
    assert np.isfinite(tl).all()
