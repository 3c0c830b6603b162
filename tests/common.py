"""Helpers shared by the GPU tests: host copies, relative L2, and training samples drawn by the
oracle in the form both sides take them (the GPU gets them as query buffers, the oracle as FP64
copies of the same FP32 values), so that no input of the oracle comes from the GPU."""
import numpy as np

import oracle


def host(t):
    return t.detach().cpu().double().numpy()


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


class Samples:
    """B training samples of one frame and step drawn by the oracle: point indices, directions
    and targets, the directions and targets rounded to FP32."""

    def __init__(self, points, lobes, B, seed, frame, step, output=0):
        idx, d, t = oracle.train_batch(points, lobes, B, seed, frame, step, output=output)
        self.idx = np.ascontiguousarray(idx, np.int32)
        self.d32 = np.ascontiguousarray(d, np.float32)
        self.t32 = np.ascontiguousarray(t, np.float32)

    @property
    def d(self):
        return self.d32.astype(np.float64)

    @property
    def t(self):
        return self.t32.astype(np.float64)

    def queries(self, nirc):
        import torch
        return nirc.Queries.from_dirs(torch.from_numpy(self.d32).cuda(), torch.from_numpy(self.idx).cuda())

    def target(self):
        import torch
        return torch.from_numpy(self.t32).cuda()

    def loss_grad(self, points, w, width):
        return oracle.loss_grad(points, self.idx, self.d, self.t, w, width)

    def select(self, keep):
        """Keep the samples where `keep` (a mask or an index array) says so."""
        self.idx = np.ascontiguousarray(self.idx[keep])
        self.d32 = np.ascontiguousarray(self.d32[keep])
        self.t32 = np.ascontiguousarray(self.t32[keep])

    def drop_relu_ties(self, points, w, width, band=1e-5):
        """Drop the samples whose hidden pre-activations come within `band` of zero (FP64, numpy
        matrix chain).  There the ReLU mask is decided by rounding: an FP32 forward pass may take
        the other side, and the one sample's flipped unit moves a gradient over a few thousand
        samples by ~1e-4.  FP32 pre-activations err by ~1e-6 at most, so 1e-5 leaves a margin.
        Returns the number of samples dropped."""
        from tests import npref
        _, pre = npref.forward(npref.encode(npref.inputs_of(points, self.idx, self.d)), w, width)
        keep = np.ones(self.idx.shape[0], bool)
        for z in pre:
            keep &= (np.abs(z) >= band).all(axis=1)
        self.select(keep)
        return int((~keep).sum())


def oracle_dirs32(points, n_cache, seed, frame):
    """The oracle's sampled directions of a frame rounded to FP32, [P * (n_cache + 1), 3]."""
    return np.ascontiguousarray(oracle.sample_dirs(points, n_cache, seed, frame).reshape(-1, 3), np.float32)


# unit roundoff of the MFMA operand format of each precision
UNIT_ROUNDOFF = {"fp32": 2.0 ** -24, "bf16": 2.0 ** -9, "fp16": 2.0 ** -12}


def relu_tie_mask(inputs, mats, u, k=8.0):
    """Samples none of whose hidden units sits within k sigma of its ReLU switch, where sigma is
    the spread that operand rounding with unit roundoff u gives the unit's pre-activation.

    inputs: [B, n] FP64 network inputs; mats: the five weight matrices (FP64).  For a unit r of
    layer l with FP64 inputs h, operands rounded independently with relative errors uniform in
    [-u, u] move z = sum_c W_rc h_c by a sum of independent terms W_rc h_c (a_c + b_c), variance
    (2/3) u^2 sum_c (W_rc h_c)^2; the error a unit carries on to the next layer (where it is on)
    adds sum_c W_rc^2 sigma_c^2.  A sample whose |z| >= k sigma at every unit is decided the same
    way by any pass whose operand roundings stay within u; the others are ties."""
    keep = np.ones(inputs.shape[0], bool)
    h, var_prev = inputs, np.zeros_like(inputs)
    for W in mats[:4]:
        z = h @ W.T
        var = (2.0 / 3.0) * u * u * ((h * h) @ (W * W).T) + var_prev @ (W * W).T
        keep &= (np.abs(z) >= k * np.sqrt(var)).all(axis=1)
        var_prev = var * (z > 0)
        h = np.maximum(z, 0.0)
    return keep


def hash_mats(w, width=64):
    from paper_2412_04634_amd import workload as wl
    w = np.asarray(w, np.float64)
    mats, o = [], 0
    for r, c in wl.hash_layer_shapes(width):
        mats.append(w[o:o + r * c].reshape(r, c))
        o += r * c
    return mats


def hash_tie_free_samples(points, lobes, B, seed, frame, step, w, grid, u, k=8.0, max_draw=2 ** 19):
    """Up to B training samples of the hash-input cache (drawn as Samples draws them, from a
    longer run of the same counters) with no hidden unit within rounding of its ReLU switch
    (relu_tie_mask), so that a pass in 16-bit operands takes every ReLU decision as the FP64
    oracle does.  Returns (samples, fraction of the candidates kept)."""
    over = 64 if u >= 2.0 ** -9 else 4 if u >= 2.0 ** -12 else 2   # kept: ~2%, ~60%, ~all
    n = int(min(max(over * B, 4096), max_draw))
    sm = Samples(points, lobes, n, seed, frame, step)
    mats = hash_mats(w)
    nm = sum(m.size for m in mats)
    table = np.asarray(w, np.float64)[nm:]
    keep = np.zeros(n, bool)
    for a in range(0, n, 65536):
        b = min(n, a + 65536)
        e = oracle.hash_encode(points, sm.idx[a:b], sm.d[a:b], table, grid)
        keep[a:b] = relu_tie_mask(e, mats, u, k)
    frac = float(keep.mean())
    sm.select(np.flatnonzero(keep)[:B])
    return sm, frac


def point_errors(got, ref, scale):
    """Per point (rows of [P, 3]): |got_p - ref_p|_2 / |scale_p|_2, where scale is a positive
    magnitude of the same point (the cache's own prediction, which has no cancellation)."""
    got = np.asarray(got, np.float64).reshape(-1, 3)
    ref = np.asarray(ref, np.float64).reshape(-1, 3)
    s = np.linalg.norm(np.asarray(scale, np.float64).reshape(-1, 3), axis=1)
    return np.linalg.norm(got - ref, axis=1) / np.maximum(s, 1e-300)


# Per-point bounds (max over points, beside the rel-L2 over the array).  A query's cache output
# y = exp(z) carries the relative error of z: in FP32 a few ulp of the layer sums (measured
# <= 1e-6 per query), in 16-bit operands the spread of operand rounding, sigma ~ 2e-3 (BF16) /
# 2.5e-4 (FP16) of z's scale, so that the worst of ~10^5 queries reaches ~5 sigma.  F_c averages
# N such errors; the residual F_r = L - y_r carries one query's error plus the field's change
# over the direction error (kappa |dw| <= 50 * 3e-7 in FP32).  Hence, relative to the point's own
# scale |F_c,p| + |y_r,p| (y_r = the oracle's prediction at the residual direction):
POINT_TOL = {"fp32": 2e-5, "bf16": 8e-3, "fp16": 2e-3}
# and for single cache outputs relative to |y_q|:
QUERY_TOL = {"fp32": 2e-5, "bf16": 1.5e-2, "fp16": 3e-3}


def check_query_points(label, y, ref, prec):
    """Per-query bound on cache outputs; returns the worst ratio."""
    e = point_errors(y, ref, ref)
    worst = float(e.max()) if e.size else 0.0
    print(f"  {label}: worst query |dy|/|y| {worst:.3e} (bound {QUERY_TOL[prec]:.1e})", flush=True)
    assert worst <= QUERY_TOL[prec], (label, worst, int(e.argmax()))
    return worst


def check_estimate_points(label, tl, c, r, o_tl, o_c, o_r, y_r, prec):
    """Per-point bounds on an estimate: F_c relative to |F_c,p|; F_r and F_tl relative to
    |F_c,p| + |y_r,p|.  y_r: [P, 3] the oracle's cache prediction at each point's residual
    direction.  Returns the worst ratios (F_c, F_r, F_tl)."""
    scale = np.linalg.norm(np.asarray(o_c).reshape(-1, 3), axis=1) + \
        np.linalg.norm(np.asarray(y_r).reshape(-1, 3), axis=1)
    s3 = np.repeat(scale[:, None], 3, axis=1) / np.sqrt(3.0)
    ec = point_errors(c, o_c, o_c)
    er = point_errors(r, o_r, s3)
    et = point_errors(tl, o_tl, s3)
    w = tuple(float(a.max()) if a.size else 0.0 for a in (ec, er, et))
    print(f"  {label}: worst point F_c {w[0]:.3e}, F_r {w[1]:.3e}, F_tl {w[2]:.3e} (bound {POINT_TOL[prec]:.1e})",
          flush=True)
    assert max(w) <= POINT_TOL[prec], (label, w, int(ec.argmax()), int(er.argmax()), int(et.argmax()))
    return w


def residual_prediction(points, w, width, n_cache, seed, frame, dirs=None, ids=None, hash_grid=None):
    """The oracle's cache prediction at each point's residual direction, [P, 3]."""
    if dirs is None:
        dirs = oracle.sample_dirs(points, n_cache, seed, frame, ids=ids)
    dr = np.ascontiguousarray(np.asarray(dirs).reshape(points.count, n_cache + 1, 3)[:, n_cache, :])
    if hash_grid is not None:
        return oracle.hash_infer(points, None, dr, w, width, hash_grid)
    return oracle.infer(points, None, dr, w, width)
