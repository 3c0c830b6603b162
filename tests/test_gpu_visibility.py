"""The visibility cache (Sec. "Neural Visibility Cache") and the occluded scene against the FP64
oracle (needs the GPU).  The visibility cache's sigmoid outputs times the known radiance form
the cache level; the residual sample and the radiance cache's targets on the occluded scene are
V L.  Tolerances as for the radiance cache: FP32 outputs and gradients rel-L2 1e-5 on the same
queries, the fused estimator's F_c 1e-5 and F_tl, F_r within 1e-5 of |F_c| against the oracle's
own directions; 16-bit operands 1e-2 (gradients ten unit roundoffs)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import Samples, host, rel_l2
from tests.common import check_query_points

pytestmark = pytest.mark.gpu
VIS, OCC = 1, 2
PRECS = {"fp32": 0, "bf16": 1}
TOL = {"fp32": 1e-5, "bf16": 1e-2}
GRAD_TOL = {"fp32": 1e-5, "bf16": 10 * 2.0 ** -9}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


@pytest.mark.parametrize("output", [VIS, OCC])
def test_train_batch_targets(nirc, output):
    P, B = 3000, 4099
    pts = wl.make_points(110, P)
    lob = wl.make_lobes(110).packed()
    dp = nirc.Points.from_workload(pts)
    q, tgt = nirc.tlmc_train_batch(dp, lob, B, 11, 2, 1, output=output)
    idx, d, t = oracle.train_batch(pts, lob, B, 11, 2, 1, output=output)
    np.testing.assert_array_equal(q.point.cpu().numpy(), idx)
    e = rel_l2(host(tgt), t)
    print(f"targets output={output} rel-L2 {e:.2e}", flush=True)
    assert e <= 1e-5


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_infer_visibility(nirc, prec):
    P, Q = 500, 4099
    pts = wl.make_points(111, P)
    w0 = wl.make_weights(111, 64)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec], output=VIS), max_batch=0)
    g = torch.Generator().manual_seed(1)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g, dtype=torch.float64)
    d = (d / d.norm(dim=1, keepdim=True)).float()
    y = host(nirc.nirc_infer(model, dp, nirc.Queries.from_dirs(d.cuda(), idx.cuda())))
    ref = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0, 64, output=VIS)
    assert rel_l2(y, ref) <= TOL[prec]
    check_query_points(f"visibility infer {prec}", y, ref, prec)
    assert (y > 0).all() and (y < 1).all()


@pytest.mark.parametrize("output", [VIS, OCC])
@pytest.mark.parametrize("prec,W,P,N", [("fp32", 64, 1000, 16), ("fp32", 64, 333, 3), ("bf16", 64, 2048, 8),
                                        ("bf16", 64, 100, 64), ("fp32", 128, 300, 8), ("bf16", 128, 200, 16)])
def test_estimate_occluded(nirc, output, prec, W, P, N):
    print(f"estimate output={output} {prec} W={W} P={P} N={N}", flush=True)
    pts = wl.make_points(112, P)
    lob = wl.make_lobes(112).packed()
    w0 = wl.make_weights(112, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(width=W, precision=PRECS[prec], output=output), max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lob, N, 13, 3, parts=True))
    o_tl, o_c, o_r = oracle.estimate(pts, lob, w0, W, N, 13, 3, output=output)
    e_c = rel_l2(c, o_c)
    e_tl = np.linalg.norm(tl - o_tl) / np.linalg.norm(o_c)
    e_r = np.linalg.norm(r - o_r) / np.linalg.norm(o_c)
    print(f"  F_c rel-L2 {e_c:.2e}; F_tl, F_r error / |F_c| {e_tl:.2e}, {e_r:.2e}", flush=True)
    assert e_c <= TOL[prec] and e_tl <= TOL[prec] and e_r <= TOL[prec]


@pytest.mark.parametrize("prec,B", [("fp32", 1000), ("fp32", 16384), ("bf16", 4096)])
def test_loss_grad_visibility(nirc, prec, B):
    P, W = 3000, 64
    pts = wl.make_points(113, P)
    lob = wl.make_lobes(113).packed()
    w0 = wl.make_weights(113, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(precision=PRECS[prec], output=VIS), max_batch=B)
    sm = Samples(pts, lob, B, 14, 0, 0, output=VIS)
    if prec == "fp32":
        sm.drop_relu_ties(pts, w0, W)
    loss, grad = nirc.nirc_loss_grad(model, dp, sm.queries(nirc), sm.target())
    o_loss, o_grad = oracle.loss_grad(pts, sm.idx, sm.d, sm.t, w0, W, output=VIS)
    e_loss = abs(float(loss.item()) - o_loss) / o_loss
    e_grad = rel_l2(host(grad), o_grad)
    print(f"visibility loss {prec} B={B}: loss rel err {e_loss:.2e} grad rel-L2 {e_grad:.2e}", flush=True)
    assert e_loss <= GRAD_TOL[prec] and e_grad <= GRAD_TOL[prec]


def test_reference_occluded_matches_oracle(nirc):
    P = 40
    pts = wl.make_points(114, P)
    lob = wl.make_lobes(114).packed()
    dp = nirc.Points.from_workload(pts)
    F = host(nirc.tlmc_reference_occluded(dp, lob, 64))
    ref64 = oracle.quadrature(pts, lob, VIS, 64)
    ref = oracle.quadrature(pts, lob, VIS, 384)
    e64, econv = rel_l2(F, ref64), rel_l2(F, ref)
    print(f"occluded reference: vs the oracle's 64-node rule {e64:.2e}, vs 384 nodes {econv:.2e}", flush=True)
    assert e64 <= 1e-5        # same rule, FP32 integrand
    assert econv <= 1e-3      # the 64-node rule's own error on these lobes


def test_biased_and_batched_visibility(nirc):
    P, N, W = 3000, 8, 64
    pts = wl.make_points(115, P)
    lob = wl.make_lobes(115).packed()
    w0 = wl.make_weights(115, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(output=VIS), max_batch=0)
    b, c, cont = (host(t) for t in nirc.tlmc_estimate_biased(model, dp, lob, N, 5, 2))
    o_b, o_cont = oracle.estimate_biased(pts, lob, w0, W, N, 5, 2, output=VIS)
    _, o_c, _ = oracle.estimate(pts, lob, w0, W, N, 5, 2, output=VIS)
    np.testing.assert_array_equal(cont, o_cont)
    go = cont == 1
    assert np.linalg.norm(b[go] - o_b[go]) <= 1e-5 * np.linalg.norm(o_c)
    # a visibility-cache request in a batch gives exactly its result alone
    out = torch.full((P, 3), -1.0, device="cuda")
    batch = nirc.Batch()
    batch.set([dict(model=model, points=dp, lobes=lob, n_cache=N, seed=5, frame=2, out_tl=out)])
    batch.launch()
    assert torch.equal(out, nirc.tlmc_estimate(model, dp, lob, N, 5, 2))


def test_train_frames_visibility(nirc):
    # three frames of four steps with the visibility cache follow the FP64 trajectory
    P, B, W = 4096, 4096, 64
    pts = wl.make_points(116, P)
    lob = wl.make_lobes(116).packed()
    w0 = wl.make_weights(116, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(output=VIS), max_batch=B)
    w = w0.astype(np.float64).copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    t = 0
    losses, o_losses = [], []
    loss = torch.zeros(1, device="cuda")
    for f in range(3):
        nirc.nirc_train_frame(model, dp, lob, B, 4, 17, f, loss)
        losses.append(float(loss.item()))
        for s in range(4):
            idx, d, tg = oracle.train_batch(pts, lob, B, 17, f, s, output=VIS)
            lo, g = oracle.loss_grad(pts, idx, d, tg, w, W, output=VIS)
            t += 1
            oracle.adam(w, m, v, g, t, lr=1e-3)
        o_losses.append(lo)
    print("  visibility losses", np.round(losses, 5), "oracle", np.round(o_losses, 5), flush=True)
    assert np.max(np.abs(np.array(losses) - o_losses) / np.array(o_losses)) <= 1e-3
    assert rel_l2(host(model.get_weights()) - w0, w - w0) <= 1e-2


def test_batch_rejects_mixed_output_modes(nirc):
    pts = nirc.Points.from_workload(wl.make_points(117, 100))
    lob = wl.make_lobes(117).packed()
    a = nirc.Model(wl.make_weights(117, 64), max_batch=0)
    b = nirc.Model(wl.make_weights(118, 64), cfg=nirc.make_config(output=VIS), max_batch=0)
    reqs = [dict(model=m, points=pts, lobes=lob, n_cache=4, seed=1, frame=0, out_tl=torch.empty((100, 3), device="cuda"))
            for m in (a, b)]
    with pytest.raises(nirc.NircError):
        nirc.Batch().set(reqs)
