"""CPU model of 16-bit training arithmetic (BF16-rounded operands, FP32 products summed in FP64)
against the FP64 oracle gradient.  It backs the batch sizes at which the GPU 16-bit gradients
are held to ten unit roundoffs: one sample's gradient can be dominated by a ReLU mask that
16-bit rounding flips, a batch's cannot."""
import numpy as np

import oracle
from paper_2412_04634_amd import workload as wl


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as FP64."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def features(pts, idx, d):
    cols = [pts.px[idx], pts.py[idx], pts.pz[idx], d[:, 0], d[:, 1], d[:, 2], pts.nx[idx], pts.ny[idx],
            pts.nz[idx], pts.rough[idx]]
    out = []
    for v in cols:
        a = np.pi * (2.0 ** np.arange(8))[None, :] * np.asarray(v, np.float64)[:, None]
        e = np.empty((a.shape[0], 16))
        e[:, 0::2], e[:, 1::2] = np.sin(a), np.cos(a)
        out.append(e)
    return np.concatenate(out, 1)


def grad_model(W, w, e, t, rounding):
    mats, o = [], 0
    for r, c in wl.layer_shapes(W):
        mats.append(w[o:o + r * c].reshape(r, c))
        o += r * c
    q = bf16 if rounding else (lambda x: x)
    hs = [q(e)]
    for l in range(4):
        hs.append(q(np.maximum(hs[-1] @ q(mats[l]).T, 0.0)))
    y = np.exp(hs[-1] @ q(mats[4]).T)
    B = y.shape[0]
    d5 = 2.0 * (y - t) * y / (y * y + 1e-2)           # per sample, before the 1 / (3B)
    grads = [None] * 5
    grads[4] = q(d5).T @ hs[4] / (3 * B)
    delta = q(d5) @ q(mats[4])
    for l in range(3, -1, -1):
        delta = q(delta * (hs[l + 1] > 0))
        grads[l] = delta.T @ hs[l] / (3 * B)
        if l > 0:
            delta = delta @ q(mats[l])
    return np.concatenate([g.ravel() for g in grads])


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_model_without_rounding_is_the_oracle_gradient():
    pts = wl.make_points(44, 3000)
    lob = wl.make_lobes(44).packed()
    w = wl.make_weights(44, 64).astype(np.float64)
    idx, d, t = oracle.train_batch(pts, lob, 200, 45, 0, 0)
    _, og = oracle.loss_grad(pts, idx, d, t, w, 64)
    assert rel(grad_model(64, w, features(pts, idx, d), t, False), og) <= 1e-9


def test_single_sample_can_exceed_the_batch_tolerance():
    tol = 10 * 2.0 ** -9
    pts = wl.make_points(44, 3000)
    lob = wl.make_lobes(44).packed()
    w = wl.make_weights(44, 128).astype(np.float64)
    errs = {}
    for B in (1, 1000):
        idx, d, t = oracle.train_batch(pts, lob, B, 45, 0, 0)
        _, og = oracle.loss_grad(pts, idx, d, t, w, 128)
        errs[B] = rel(grad_model(128, w, features(pts, idx, d), t, True), og)
    assert errs[1] > tol        # a flipped mask: one sample's gradient is off by far more
    assert errs[1000] <= tol / 2


def fp16(x):
    return np.asarray(x, np.float32).astype(np.float16).astype(np.float64)


def test_first_layer_error_is_magnified_but_bounded(monkeypatch):
    # the first layer's gradient sums cancelling per-sample terms, so its relative rounding error
    # is several times the whole gradient's; at B = 1000 it stays below the 0.1 per-layer bound
    import tests.test_precision_model as m
    pts = wl.make_points(44, 3000)
    lob = wl.make_lobes(44).packed()
    w = wl.make_weights(44, 128).astype(np.float64)
    idx, d, t = oracle.train_batch(pts, lob, 1000, 45, 0, 0)
    _, og = oracle.loss_grad(pts, idx, d, t, w, 128)
    n1 = 128 * 160
    for rounding, tol in ((bf16, 10 * 2.0 ** -9), (fp16, 10 * 2.0 ** -12)):
        monkeypatch.setattr(m, "bf16", rounding)
        g = m.grad_model(128, w, features(pts, idx, d), t, True)
        e_all, e_w1 = rel(g, og), rel(g[:n1], og[:n1])
        assert e_all <= tol
        assert e_all < e_w1 < 0.1
