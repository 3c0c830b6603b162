"""Width-128 caches (the precision form's second width) against the FP64 oracle (needs the GPU).

Same tolerances as at width 64: FP32 rel-L2 <= 1e-5 on the same directions, 16-bit operands
rel-L2 <= 1e-2.  Training at width 128 is reported as unsupported.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl

pytestmark = pytest.mark.gpu
W = 128
PRECS = {"fp32": 0, "bf16": 1, "fp16": 2}
TOL = {"fp32": 1e-5, "bf16": 1e-2, "fp16": 1e-2}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


def host(t):
    return t.detach().cpu().double().numpy()


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def test_parameter_count(nirc):
    assert nirc.nirc_n_params(W) == W * 160 + 3 * W * W + 3 * W == 70016


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("Q", [1, 1000, 4099])
def test_infer_width128(nirc, prec, Q):
    print(f"infer W=128 {prec} Q={Q}", flush=True)
    P = 400
    pts = wl.make_points(41, P)
    w0 = wl.make_weights(41, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(width=W, precision=PRECS[prec]), max_batch=0)
    g = torch.Generator().manual_seed(Q)
    idx = torch.randint(0, P, (Q,), generator=g, dtype=torch.int32)
    d = torch.randn(Q, 3, generator=g, dtype=torch.float64)
    d = (d / d.norm(dim=1, keepdim=True).clamp_min(1e-9)).float()
    y = host(nirc.nirc_infer(model, dp, nirc.Queries.from_dirs(d.cuda(), idx.cuda())))
    ref = oracle.infer(pts, idx.numpy(), d.double().numpy(), w0, W)
    assert rel_l2(y, ref) <= TOL[prec]


@pytest.mark.parametrize("prec", ["fp32", "bf16", "fp16"])
@pytest.mark.parametrize("P,N", [(17, 3), (4096, 4), (1000, 16), (100, 64)])
def test_estimate_width128(nirc, prec, P, N):
    print(f"estimate W=128 {prec} P={P} N={N}", flush=True)
    pts = wl.make_points(42, P)
    lob = wl.make_lobes(42).packed()
    w0 = wl.make_weights(42, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(width=W, precision=PRECS[prec]), max_batch=0)
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, lob, N, 11, 2, parts=True))
    dirs = host(nirc.tlmc_sample_dirs(dp, N, 11, 2))
    o_tl, o_c, o_r = oracle.estimate(pts, lob, w0, W, N, 11, 2, dirs=dirs)
    assert rel_l2(c, o_c) <= TOL[prec]
    assert rel_l2(tl, o_tl) <= TOL[prec]
    assert np.linalg.norm(r - o_r) <= TOL[prec] * np.linalg.norm(o_c)


def test_training_width128_unsupported(nirc):
    P, B = 500, 256
    pts = wl.make_points(43, P)
    lob = wl.make_lobes(43).packed()
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(wl.make_weights(43, W), cfg=nirc.make_config(width=W), max_batch=B)
    q, tgt = nirc.tlmc_train_batch(dp, lob, B, 1, 0, 0)
    with pytest.raises(nirc.NircError, match="unsupported"):
        nirc.nirc_train_step(model, dp, q, tgt)
