"""The estimator's residual radiance input and the state blob (needs the GPU).

Residual radiance (a renderer's path-traced sample at the residual direction): with R given,
F_r = R - n(x, w_r) and F_c is untouched.  Checked against the oracle (its own directions:
F_r within 1e-5 of |F_c| in FP32, 1e-2 for 16-bit operands), against the field path when R is
the field at the oracle's residual directions, and in a batched launch (bitwise equal to the
same request alone).

State blob: a model restored from another's blob continues bit for bit as the saved one.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2412_04634_amd import workload as wl
from tests.common import Samples, host
from tests.common import check_estimate_points

pytestmark = pytest.mark.gpu
PRECS = {"fp32": 0, "bf16": 1, "fp16": 2}
EST_TOL = {"fp32": 1e-5, "bf16": 1e-2, "fp16": 1e-2}


@pytest.fixture(scope="module")
def nirc():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2412_04634_amd import nirc as m
    m.lib()
    return m


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("W,P,N", [(64, 1000, 16), (64, 17, 3), (128, 300, 8), (128, 100, 16)])
def test_estimate_with_residual_radiance(nirc, prec, W, P, N):
    print(f"residual radiance {prec} W={W} P={P} N={N}", flush=True)
    pts = wl.make_points(60, P)
    lob = wl.make_lobes(60).packed()
    w0 = wl.make_weights(60, W)
    dp = nirc.Points.from_workload(pts)
    model = nirc.Model(w0, cfg=nirc.make_config(width=W, precision=PRECS[prec]), max_batch=0)
    seed, frame = 61, 4
    rng = np.random.default_rng(62)
    R = rng.uniform(0.0, 3.0, (P, 3)).astype(np.float32)
    Rd = torch.from_numpy(R).cuda()
    tl, c, r = (host(t) for t in nirc.tlmc_estimate(model, dp, None, N, seed, frame, parts=True, residual=Rd))
    tl_f, c_f, r_f = (host(t) for t in nirc.tlmc_estimate(model, dp, lob, N, seed, frame, parts=True))
    np.testing.assert_array_equal(c, c_f)            # the cache level does not read the residual
    np.testing.assert_allclose(tl, c + r, rtol=0, atol=4e-7 * np.abs(tl).max())   # F_tl = F_c + F_r in FP32
    # oracle: n(x, w_r) at its own residual directions and its own F_c
    dirs = oracle.sample_dirs(pts, N, seed, frame)
    y_r = oracle.infer(pts, np.arange(P, dtype=np.int32), dirs[:, N, :], w0, W)
    _, o_c, _ = oracle.estimate(pts, lob, w0, W, N, seed, frame, dirs=dirs)
    e_r = np.linalg.norm(r - (R - y_r)) / np.linalg.norm(o_c)
    print(f"  F_r error / |F_c| {e_r:.2e}", flush=True)
    assert e_r <= EST_TOL[prec]
    # per point: F_c, and F_r = R - y_r relative to |F_c,p| + |y_r,p|
    check_estimate_points(f"residual tile {prec} W={W}", tl, c, r, o_c + (R - y_r), o_c, R - y_r, y_r,
                          prec)
    # R = the field at the oracle's residual directions reproduces the field path
    Lf = oracle.field(lob, pts, None, dirs[:, N, :]).astype(np.float32)
    tl2 = host(nirc.tlmc_estimate(model, dp, None, N, seed, frame, residual=torch.from_numpy(Lf).cuda()))
    assert np.linalg.norm(tl2 - tl_f) <= 1e-5 * np.linalg.norm(c_f)


def test_batched_request_with_residual_radiance(nirc):
    print("batched residual radiance", flush=True)
    reqs, alone = [], []
    for i, (P, N) in enumerate([(3000, 8), (17, 4), (4096, 16)]):
        pts = nirc.Points.from_workload(wl.make_points(70 + i, P))
        model = nirc.Model(wl.make_weights(70 + i, 64), cfg=nirc.make_config(precision=1), max_batch=0)
        R = torch.from_numpy(np.random.default_rng(i).uniform(0, 2, (P, 3)).astype(np.float32)).cuda()
        lob = wl.make_lobes(70 + i).packed()
        rr = R if i != 1 else None          # one request on the field
        reqs.append(dict(model=model, points=pts, lobes=None if rr is not None else lob, n_cache=N, seed=9 + i,
                         frame=i, residual=rr, out_tl=torch.full((P, 3), -1.0, device="cuda")))
        alone.append(nirc.tlmc_estimate(model, pts, None if rr is not None else lob, N, 9 + i, i, residual=rr))
    b = nirc.Batch()
    b.set(reqs)
    b.launch()
    for r, a in zip(reqs, alone):
        assert torch.equal(r["out_tl"], a)


def test_residual_radiance_argument_errors(nirc):
    pts = nirc.Points.from_workload(wl.make_points(80, 10))
    model = nirc.Model(wl.make_weights(80, 64), max_batch=0)
    with pytest.raises(nirc.NircError):
        nirc.tlmc_estimate(model, pts, None, 4, 0, 0)   # neither field nor residual radiance


@pytest.mark.parametrize("prec,W", [("fp32", 64), ("bf16", 64), ("fp16", 128)])
def test_state_blob_resume(nirc, prec, W):
    print(f"state blob {prec} W={W}", flush=True)
    P, B = 2000, 1024
    pts = wl.make_points(81, P)
    lob = wl.make_lobes(81).packed()
    dp = nirc.Points.from_workload(pts)
    cfg = nirc.make_config(width=W, precision=PRECS[prec])
    a = nirc.Model(wl.make_weights(81, W), cfg=cfg, max_batch=B)
    for f in range(2):
        nirc.nirc_train_frame(a, dp, lob, B, 3, 82, f)
    blob = a.get_state()
    saved = host(blob.view(torch.float32)) if blob.numel() % 4 == 0 else None
    # a model with other weights takes the blob and then trains exactly as the original
    b = nirc.Model(wl.make_weights(83, W), cfg=cfg, max_batch=B)
    b.set_state(blob)
    for m in (a, b):
        nirc.nirc_train_frame(m, dp, lob, B, 3, 82, 2)
    np.testing.assert_array_equal(host(a.get_weights()), host(b.get_weights()))
    for x, y in zip(a.get_adam(), b.get_adam()):
        np.testing.assert_array_equal(host(x), host(y))
    np.testing.assert_array_equal(host(nirc.tlmc_estimate(a, dp, lob, 8, 1, 3)),
                                  host(nirc.tlmc_estimate(b, dp, lob, 8, 1, 3)))
    # the blob itself is untouched by the restore, and a blob of another size is refused
    if saved is not None:
        np.testing.assert_array_equal(host(blob.view(torch.float32)), saved)
    other = nirc.Model(wl.make_weights(84, 64 if W == 128 else 128),
                       cfg=nirc.make_config(width=64 if W == 128 else 128), max_batch=0)
    with pytest.raises(nirc.NircError):
        other.set_state(blob)
    # a gradient on oracle-drawn samples is the same on the restored model
    sm = Samples(pts, lob, 512, 85, 0, 0)
    ga = nirc.nirc_loss_grad(a, dp, sm.queries(nirc), sm.target())[1]
    gb = nirc.nirc_loss_grad(b, dp, sm.queries(nirc), sm.target())[1]
    assert torch.equal(ga, gb)
