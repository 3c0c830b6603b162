"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics (CPU only).

Each test checks the oracle against something other than itself: published known-answer
vectors, closed forms, exact special values, library routines, invariants and brute force.
"""
import decimal
import math

import numpy as np
import pytest
import scipy.integrate
import scipy.special
import scipy.stats

import oracle
from paper_2412_04634_amd import workload as wl
from tests import npref


# ------------------------------------------------------------------------------------------
# Philox4x32-10 (Salmon et al. SC'11), known-answer vectors

def test_philox_known_answers(kat_vectors):
    assert len(kat_vectors) >= 3
    for ctr, key, expect in kat_vectors:
        got = oracle.philox(ctr, key)
        assert [int(x) for x in got] == expect


# ------------------------------------------------------------------------------------------
# Frequency encoding: exact special values, library sin/cos, norm invariant

def _pts1(vals):
    """A one-point workload whose 7 point inputs all equal vals[0..6]."""
    a = [np.array([v], np.float32) for v in vals]
    return wl.Points(*a)


@pytest.mark.parametrize("v,sin_expect,cos_expect", [
    (0.0, [0] * 8, [1] * 8),
    (0.5, [1, 0, 0, 0, 0, 0, 0, 0], [0, -1, 1, 1, 1, 1, 1, 1]),
    (1.0, [0] * 8, [-1, 1, 1, 1, 1, 1, 1, 1]),
    (-0.5, [-1, 0, 0, 0, 0, 0, 0, 0], [0, -1, 1, 1, 1, 1, 1, 1]),
])
def test_encoding_exact_special_values(v, sin_expect, cos_expect):
    pts = _pts1([v] * 7)
    feat = oracle.encode(pts, None, np.array([[v, v, v]]))[0]
    for i in range(10):
        assert list(feat[16 * i:16 * i + 16:2]) == [float(s) for s in sin_expect]
        assert list(feat[16 * i + 1:16 * i + 16:2]) == [float(c) for c in cos_expect]


def test_encoding_matches_library_sin_cos_and_norm():
    rng = np.random.default_rng(7)
    pts = wl.make_points(11, 300)
    dirs = rng.normal(size=(300, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    feat = oracle.encode(pts, None, dirs)
    ref = npref.encode(npref.inputs_of(pts, None, dirs))
    np.testing.assert_allclose(feat, ref, rtol=0, atol=2e-13)
    np.testing.assert_allclose((feat ** 2).sum(axis=1), 80.0, rtol=0, atol=1e-12)


# ------------------------------------------------------------------------------------------
# MLP: numpy matrix chain, exp head with zero last layer, positive homogeneity

@pytest.mark.parametrize("width", [64, 128])
def test_mlp_matches_numpy_matrix_chain(width):
    rng = np.random.default_rng(3)
    pts = wl.make_points(5, 64)
    dirs = rng.normal(size=(64, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    w = wl.make_weights(9, width)
    got = oracle.infer(pts, None, dirs, w, width)
    ref, _ = npref.forward(npref.encode(npref.inputs_of(pts, None, dirs)), w, width)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=0)


def test_mlp_zero_output_layer_gives_one():
    width = 64
    w = wl.make_weights(2, width).copy()
    w[-3 * width:] = 0.0
    pts = wl.make_points(3, 50)
    dirs = oracle.sample_dirs(pts, 1, 1, 0)[:, 0, :]
    y = oracle.infer(pts, None, dirs, w, width)
    assert np.all(y == 1.0)


def test_mlp_relu_positive_homogeneity():
    # scaling a hidden layer by c > 0 scales the output pre-activation by c: y(cW3) = y(W)^c
    width = 64
    w = wl.make_weights(4, width).astype(np.float64)
    pts = wl.make_points(6, 40)
    dirs = oracle.sample_dirs(pts, 1, 2, 0)[:, 0, :]
    y = oracle.infer(pts, None, dirs, w, width)
    w2 = w.copy()
    off = width * 160 + width * width          # start of W3
    w2[off:off + width * width] *= 2.5
    y2 = oracle.infer(pts, None, dirs, w2, width)
    np.testing.assert_allclose(y2, y ** 2.5, rtol=1e-11)


# ------------------------------------------------------------------------------------------
# Cosine-weighted sampling: moments, hemisphere, unit length, Philox-word mapping

def test_cosine_sampler_moments():
    pts = wl.make_points(8, 64)
    n_cache = 64
    d = oracle.sample_dirs(pts, n_cache, 123, 7)            # [P, N+1, 3]
    nrm = np.stack([pts.nx, pts.ny, pts.nz], axis=1).astype(np.float64)
    nlen = np.linalg.norm(nrm, axis=1)
    # the basis is orthonormal for a unit normal; stored normals are FP32-rounded unit vectors
    np.testing.assert_allclose(np.linalg.norm(d, axis=2), 1.0, rtol=0, atol=5e-7)
    cos = np.einsum("pkd,pd->pk", d, nrm) / nlen[:, None] ** 2
    assert cos.min() >= 0.0
    c = cos.ravel()
    # cos(theta) of a cosine-weighted sample: E = 2/3, E[cos^2] = 1/2, Var = 1/18
    se = math.sqrt(1.0 / 18.0 / c.size)
    assert abs(c.mean() - 2.0 / 3.0) < 5 * se
    se2 = math.sqrt((1.0 / 3.0 - 0.25) / c.size)             # Var[cos^2] = E[cos^4]-1/4 = 1/12
    assert abs((c ** 2).mean() - 0.5) < 5 * se2
    # the mean direction is (2/3) n
    m = (d / nlen[:, None, None]).mean(axis=1)               # per-point mean over samples
    proj = np.einsum("pd,pd->p", m, nrm / nlen[:, None])
    assert abs(proj.mean() - 2.0 / 3.0) < 5 * math.sqrt(1.0 / 18.0 / (64 * 65))


def test_cosine_direction_from_philox_words():
    # direction k of point p: uniforms (r>>8)/2^24 from Philox(ctr=(p, k>>1, frame, 3)), words
    # (0,1) for even k and (2,3) for odd k; the local frame's z axis is the normal, so n.w is
    # sqrt(1-u1) whatever basis is chosen.  Residual directions of points p, p+1 (p even) share
    # counter (p/2, 0, frame, 4).
    pts = wl.make_points(21, 5)
    seed, frame = 0x1234_5678_9ABC, 3
    d = oracle.sample_dirs(pts, 4, seed, frame)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for p in range(5):
        n = np.array([pts.nx[p], pts.ny[p], pts.nz[p]], np.float64)
        for k in range(4):
            r = oracle.philox([p, k >> 1, frame, 3], key)
            u1 = (int(r[2 * (k & 1)]) >> 8) / 2.0 ** 24
            assert abs(d[p, k] @ n / (n @ n) - math.sqrt(1 - u1)) < 1e-7
        r = oracle.philox([p >> 1, 0, frame, 4], key)
        u1 = (int(r[2 * (p & 1)]) >> 8) / 2.0 ** 24
        assert abs(d[p, 4] @ n / (n @ n) - math.sqrt(1 - u1)) < 1e-7


# ------------------------------------------------------------------------------------------
# Lobe field: record layout and special directions

def test_field_special_directions():
    lobes = wl.make_lobes(3)
    rec = lobes.packed()
    pts = wl.make_points(4, 3)
    for j in range(4):
        # isolate lobe j by zeroing the other amplitudes
        iso = wl.Lobes(lobes.axis.copy(), lobes.kappa.copy(), np.zeros_like(lobes.alpha),
                       np.zeros_like(lobes.beta))
        iso.alpha[j] = lobes.alpha[j]
        iso.beta[j] = lobes.beta[j]
        mu = lobes.axis[j].astype(np.float64)
        for p in range(3):
            x = np.array([pts.px[p], pts.py[p], pts.pz[p]], np.float64)
            amp = lobes.alpha[j].astype(np.float64) + lobes.beta[j].astype(np.float64) @ x
            dirs = np.stack([mu, -mu])
            L = oracle.field(iso.packed(), pts, np.array([p, p], np.int32), dirs)
            mm = mu @ mu
            np.testing.assert_allclose(L[0], amp * math.exp(lobes.kappa[j] * (mm - 1)), rtol=1e-12)
            np.testing.assert_allclose(L[1], amp * math.exp(lobes.kappa[j] * (-mm - 1)), rtol=1e-12)
    # the full field is the sum of the isolated lobes
    d = oracle.sample_dirs(pts, 2, 5, 0).reshape(-1, 3)
    idx = np.repeat(np.arange(3), 3).astype(np.int32)
    total = oracle.field(rec, pts, idx, d)
    acc = 0
    for j in range(4):
        iso = wl.Lobes(lobes.axis, lobes.kappa, np.zeros_like(lobes.alpha), np.zeros_like(lobes.beta))
        iso.alpha = lobes.alpha.copy() * (np.arange(4) == j)[:, None]
        iso.beta = lobes.beta.copy() * (np.arange(4) == j)[:, None, None]
        acc = acc + oracle.field(iso.packed(), pts, idx, d)
    np.testing.assert_allclose(total, acc, rtol=1e-13)


# ------------------------------------------------------------------------------------------
# Bessel I0, Gauss-Legendre, closed-form J

@pytest.mark.parametrize("z", [0.0, 1e-3, 0.5, 1.0, 3.7, 10.0, 25.0, 49.9])
def test_bessel_i0_matches_scipy(z):
    assert oracle.bessel_i0(z) == pytest.approx(float(scipy.special.i0(z)), rel=1e-13)


def test_gauss_legendre_exact_on_polynomials():
    x, w = oracle.gauss_legendre(16)
    for k in range(0, 32):
        assert (w * x ** k).sum() == pytest.approx(1.0 / (k + 1), rel=1e-13)


def _J_t1(k):
    return 2 * math.exp(-k) * (math.exp(k) * (k - 1) + 1) / k ** 2


def _J_tm1(k):
    return 2 * math.exp(-k) * (1 - math.exp(-k) * (1 + k)) / k ** 2


@pytest.mark.parametrize("kappa", [5.0, 17.3, 50.0])
def test_J_elementary_limits(kappa):
    assert oracle.J(kappa, 1.0) == pytest.approx(_J_t1(kappa), rel=1e-13)
    assert oracle.J(kappa, -1.0) == pytest.approx(_J_tm1(kappa), rel=1e-11, abs=1e-300)


@pytest.mark.parametrize("kappa,t", [(5.0, 0.3), (50.0, -0.6), (12.0, 0.0), (33.0, 0.95)])
def test_J_full_sphere_identity_and_node_count(kappa, t):
    full = 4 * t * math.exp(-kappa) * (kappa * math.cosh(kappa) - math.sinh(kappa)) / kappa ** 2
    assert oracle.J(kappa, t) - oracle.J(kappa, -t) == pytest.approx(full, rel=1e-12, abs=1e-15)
    assert oracle.J(kappa, t, 512) == pytest.approx(oracle.J(kappa, t, 256), rel=1e-13, abs=1e-300)


def test_J_small_kappa_limit():
    for t in (-0.7, 0.0, 0.4, 1.0):
        assert oracle.J(1e-6, t) == pytest.approx(1.0, abs=1e-5)


@pytest.mark.parametrize("kappa,t", [(5.0, 0.3), (20.0, -0.2), (8.0, 0.9)])
def test_J_two_dimensional_brute_force(kappa, t):
    # (1/pi) int_{H+} exp(kappa (mu.w - 1)) cos(theta) dw over (theta, phi) with scipy dblquad
    s = math.sqrt(1 - t * t)

    def f(phi, th):
        mw = s * math.sin(th) * math.cos(phi) + t * math.cos(th)
        return math.exp(kappa * (mw - 1)) * math.cos(th) * math.sin(th)

    val, err = scipy.integrate.dblquad(f, 0, math.pi / 2, 0, 2 * math.pi, epsabs=1e-13, epsrel=1e-11)
    assert oracle.J(kappa, t) == pytest.approx(val / math.pi, rel=1e-9)


def test_second_moment_against_quadrature():
    # E[L^2] by the lobe-product closed form vs a deterministic hemisphere quadrature of L^2
    pts = wl.make_points(22, 6)
    lobes = wl.make_lobes(22).packed()
    M2 = oracle.second_moment(pts, lobes)
    gx, gw = np.polynomial.legendre.leggauss(400)
    u1 = 0.5 * (gx + 1)
    wu = 0.5 * gw
    m2 = 400
    u2 = (np.arange(m2) + 0.5) / m2
    U1, U2 = np.meshgrid(u1, u2, indexing="ij")
    Wt = np.outer(wu, np.full(m2, 1.0 / m2)).ravel()
    for p in range(6):
        nrm = np.array([pts.nx[p], pts.ny[p], pts.nz[p]], np.float64)
        nrm /= np.linalg.norm(nrm)
        a = np.array([1.0, 0, 0]) if abs(nrm[0]) < 0.9 else np.array([0, 1.0, 0])
        t1 = np.cross(nrm, a); t1 /= np.linalg.norm(t1)
        t2 = np.cross(nrm, t1)
        r = np.sqrt(U1.ravel())
        loc = np.stack([r * np.cos(2 * np.pi * U2.ravel()), r * np.sin(2 * np.pi * U2.ravel()),
                        np.sqrt(1 - U1.ravel())], axis=1)
        dirs = loc[:, :1] * t1 + loc[:, 1:2] * t2 + loc[:, 2:3] * nrm
        L = oracle.field(lobes, pts, np.full(dirs.shape[0], p, np.int32), dirs)
        q = (Wt[:, None] * L * L).sum(0)
        np.testing.assert_allclose(M2[p], q, rtol=2e-4)
    # kappa -> 0 with a single lobe: E[L^2] = a^2 exactly (J(0, t) = 1)
    iso = wl.make_lobes(22)
    iso.kappa[:] = 0.0
    iso.alpha[1:] = 0.0
    iso.beta[:] = 0.0
    M0 = oracle.second_moment(pts, iso.packed())
    np.testing.assert_allclose(M0, np.tile(iso.alpha[0].astype(np.float64) ** 2, (6, 1)), rtol=1e-12)


def test_closed_form_against_plug_in_monte_carlo():
    # With the field itself as the cache (y := L), F_c is a plain cosine-weighted MC estimate
    # of F; its mean over many directions must reach the closed form within sampling error.
    pts = wl.make_points(12, 32)
    lobes = wl.make_lobes(12).packed()
    F = oracle.closed_form(pts, lobes)
    n_cache = 4096
    _, Fc, Fr = oracle.estimate(pts, lobes, None, 64, n_cache, 99, 0, plug_in=True)
    assert np.all(Fr == 0.0)
    d = oracle.sample_dirs(pts, n_cache, 99, 0)[:, :n_cache, :]
    idx = np.repeat(np.arange(32), n_cache).astype(np.int32)
    L = oracle.field(lobes, pts, idx, d.reshape(-1, 3)).reshape(32, n_cache, 3)
    se = L.std(axis=1, ddof=1) / math.sqrt(n_cache)
    z = (Fc - F) / se
    assert np.abs(z).max() < 5.0
    np.testing.assert_allclose(Fc, L.mean(axis=1), rtol=1e-12)


# ------------------------------------------------------------------------------------------
# Two-level estimator: special cases and unbiasedness

def test_estimator_zero_output_layer():
    width = 64
    pts = wl.make_points(13, 40)
    lobes = wl.make_lobes(13).packed()
    w = wl.make_weights(13, width).astype(np.float64)
    w[-3 * width:] = 0.0
    tl, c, r = oracle.estimate(pts, lobes, w, width, 8, 5, 2)
    assert np.all(c == 1.0)
    d = oracle.sample_dirs(pts, 8, 5, 2)[:, 8, :]
    L = oracle.field(lobes, pts, None, d)
    np.testing.assert_allclose(r, L - 1.0, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(tl, L, rtol=1e-14, atol=1e-15)


def test_estimator_decomposition_on_explicit_dirs():
    # F_c is the mean of the cache at the N cache directions; F_r is L - y at the residual one.
    width = 64
    pts = wl.make_points(14, 16)
    lobes = wl.make_lobes(14).packed()
    w = wl.make_weights(14, width)
    n = 6
    d = oracle.sample_dirs(pts, n, 77, 1)
    tl, c, r = oracle.estimate(pts, lobes, w, width, n, 77, 1)
    tl2, c2, r2 = oracle.estimate(pts, lobes, w, width, n, 0, 0, dirs=d)
    np.testing.assert_array_equal(tl, tl2)
    idx = np.repeat(np.arange(16), n + 1).astype(np.int32)
    y = npref.forward(npref.encode(npref.inputs_of(pts, idx, d.reshape(-1, 3))), w, width)[0]
    y = y.reshape(16, n + 1, 3)
    L = oracle.field(lobes, pts, None, d[:, n, :])
    np.testing.assert_allclose(c, y[:, :n].mean(axis=1), rtol=1e-12)
    np.testing.assert_allclose(r, L - y[:, n], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(tl, c + r, rtol=1e-15)


@pytest.mark.parametrize("kind", ["random", "zero_out", "scaled"])
def test_estimator_unbiased_over_seeds(kind):
    # E[F_tl] = F for any cache weights (two-level MC is unbiased); z-test over S seeds
    width = 64
    P, n, S = 12, 4, 400
    pts = wl.make_points(15, P)
    lobes = wl.make_lobes(15).packed()
    w = wl.make_weights(15, width).astype(np.float64)
    if kind == "zero_out":
        w[-3 * width:] = 0.0
    if kind == "scaled":
        w[-3 * width:] *= 3.0
    F = oracle.closed_form(pts, lobes)
    samples = np.stack([oracle.estimate(pts, lobes, w, width, n, 1000 + s, 0)[0] for s in range(S)])
    mean = samples.mean(axis=0)
    se = samples.std(axis=0, ddof=1) / math.sqrt(S)
    z = (mean - F) / se
    assert np.abs(z).max() < 4.5, (kind, np.abs(z).max())


def test_estimator_mean_and_variance_match_quadrature():
    # On a tiny input, E[F_c] = (1/pi) int y cos dw and Var[F_tl] = Var[y]/N + Var[L - y]
    # (cache and residual directions are independent), both by deterministic quadrature.
    width = 64
    pts = wl.make_points(16, 1)
    lobes = wl.make_lobes(16).packed()
    w = wl.make_weights(16, width)
    n = 4
    # quadrature in the local frame: u1 = 1 - cos^2 theta is uniform for cosine sampling
    m1, m2 = 128, 128
    gx, gw = np.polynomial.legendre.leggauss(m1)
    u1 = 0.5 * (gx + 1)
    wu = 0.5 * gw
    u2 = (np.arange(m2) + 0.5) / m2
    U1, U2 = np.meshgrid(u1, u2, indexing="ij")
    W = np.outer(wu, np.full(m2, 1.0 / m2)).ravel()
    nrm = np.array([pts.nx[0], pts.ny[0], pts.nz[0]], np.float64)
    # any orthonormal frame works for the quadrature
    a = np.array([1.0, 0, 0]) if abs(nrm[0]) < 0.9 else np.array([0, 1.0, 0])
    t1 = np.cross(nrm, a); t1 /= np.linalg.norm(t1)
    t2 = np.cross(nrm, t1)
    r = np.sqrt(U1.ravel())
    loc = np.stack([r * np.cos(2 * np.pi * U2.ravel()), r * np.sin(2 * np.pi * U2.ravel()),
                    np.sqrt(1 - U1.ravel())], axis=1)
    dirs = loc[:, :1] * t1 + loc[:, 1:2] * t2 + loc[:, 2:3] * nrm
    idx = np.zeros(dirs.shape[0], np.int32)
    y = oracle.infer(pts, idx, dirs, w, width)
    L = oracle.field(lobes, pts, idx, dirs)
    Ey = (W[:, None] * y).sum(0)
    var_y = (W[:, None] * y ** 2).sum(0) - Ey ** 2
    Ed = (W[:, None] * (L - y)).sum(0)
    var_d = (W[:, None] * (L - y) ** 2).sum(0) - Ed ** 2
    S = 6000
    tl = np.zeros((S, 3))
    c = np.zeros((S, 3))
    for s in range(S):
        a_, b_, _ = oracle.estimate(pts, lobes, w, width, n, 50_000 + s, 0)
        tl[s], c[s] = a_[0], b_[0]
    var_tl = var_y / n + var_d
    assert np.all(np.abs(c.mean(0) - Ey) < 5 * np.sqrt(var_y / n / S))
    # sample variance of S draws: relative standard error ~ sqrt(2/S) (kurtosis-robust margin)
    np.testing.assert_allclose(tl.var(axis=0, ddof=1), var_tl, rtol=0.15)


# ------------------------------------------------------------------------------------------
# Loss gradient: central finite differences with a frozen denominator

def _frozen_loss(pts, idx, dirs, target, w, width, den):
    feat = npref.encode(npref.inputs_of(pts, idx, dirs))
    y, pre = npref.forward(feat, w, width)
    return ((y - target) ** 2 / den).sum() / (3.0 * y.shape[0]), pre


def test_gradient_finite_differences_frozen_denominator():
    width = 64
    B = 6
    pts = wl.make_points(17, 32)
    lobes = wl.make_lobes(17).packed()
    w = wl.make_weights(17, width).astype(np.float64)
    idx, dirs, target = oracle.train_batch(pts, lobes, B, 5, 0, 0)
    eps_l = 1e-2
    loss, g = oracle.loss_grad(pts, idx, dirs, target, w, width, eps_l, frozen=True)
    feat = npref.encode(npref.inputs_of(pts, idx, dirs))
    y0, pre0 = npref.forward(feat, w, width)
    den = y0 ** 2 + eps_l
    assert loss == pytest.approx(((y0 - target) ** 2 / den).sum() / (3 * B), rel=1e-12)
    rng = np.random.default_rng(0)
    n = w.shape[0]
    check = rng.choice(n, 300, replace=False)
    check = np.concatenate([check, np.arange(n - 3 * width, n - 3 * width + 20)])  # output layer
    h = 1e-3
    used = 0
    for i in check:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        lp, prep = _frozen_loss(pts, idx, dirs, target, wp, width, den)
        lm, prem = _frozen_loss(pts, idx, dirs, target, wm, width, den)
        if any(np.any((a > 0) != (b > 0)) or np.any((a > 0) != (c > 0)) for a, b, c in zip(pre0, prep, prem)):
            continue    # a ReLU mask flips inside the stencil: FD is not valid there
        fd = (lp - lm) / (2 * h)
        scale = max(abs(fd), 1e-6 * np.abs(g).max())
        assert abs(fd - g[i]) <= 1e-5 * scale + 1e-10, (i, fd, g[i])
        used += 1
    assert used > 250


def test_gradient_stop_gradient_is_honoured():
    # Control: differentiating through the denominator gives a different gradient, and the
    # oracle's unfrozen variant matches finite differences of the plain loss value.
    width = 64
    B = 5
    pts = wl.make_points(18, 16)
    lobes = wl.make_lobes(18).packed()
    w = wl.make_weights(18, width).astype(np.float64)
    idx, dirs, target = oracle.train_batch(pts, lobes, B, 6, 0, 0)
    _, g_frozen = oracle.loss_grad(pts, idx, dirs, target, w, width, frozen=True)
    _, g_free = oracle.loss_grad(pts, idx, dirs, target, w, width, frozen=False)
    out = slice(w.shape[0] - 3 * width, w.shape[0])
    assert np.linalg.norm(g_frozen[out] - g_free[out]) > 1e-3 * np.linalg.norm(g_frozen[out])
    h = 1e-4
    for i in range(w.shape[0] - 3 * width, w.shape[0] - 3 * width + 12):
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        lp, _ = oracle.loss_grad(pts, idx, dirs, target, wp, width, frozen=False, want_grad=False)
        lm, _ = oracle.loss_grad(pts, idx, dirs, target, wm, width, frozen=False, want_grad=False)
        fd = (lp - lm) / (2 * h)
        assert fd == pytest.approx(g_free[i], rel=1e-6, abs=1e-12)


# ------------------------------------------------------------------------------------------
# Visibility cache (Sec. "Neural Visibility Cache"): sigmoid outputs times the known radiance

def test_quadrature_reference_matches_closed_form():
    # the tensor Gauss-Legendre reference used for the occluded workload, on the unoccluded
    # field, against the closed form (independent: Bessel-function integral).  They agree to
    # 1.6e-7, not further: the closed form takes the FP32 lobe axes as exact unit vectors, the
    # field evaluation uses mu . w as stored (|mu| = 1 +- 6e-8, times kappa <= 50)
    pts = wl.make_points(23, 6)
    lobes = wl.make_lobes(23).packed()
    q = oracle.quadrature(pts, lobes, oracle.OUTPUT_RADIANCE, 384)
    F = oracle.closed_form(pts, lobes)
    assert np.abs(q - F).max() <= 4e-7 * np.abs(F).max()


def test_visibility_special_values():
    lob = wl.make_lobes(24)
    packed = lob.packed()
    mu = np.asarray(lob.axis[0], np.float64)
    perp = np.cross(mu, [1.0, 0.0, 0.0] if abs(mu[0]) < 0.9 else [0.0, 1.0, 0.0])
    perp /= np.linalg.norm(perp)
    pts = wl.Points(*[np.full(2, 0.5, np.float32) for _ in range(7)])
    v = oracle.visibility(packed, pts, None, np.stack([mu, perp]))
    sig = lambda t: 1.0 / (1.0 + math.exp(-t))
    # (the FP32 axis is a unit vector to 1e-7, so mu . mu = 1 to that accuracy)
    assert v[0] == pytest.approx(1.0 - 0.9 * sig(16.0 * (1.0 - 0.6)), rel=1e-7)
    assert v[1] == pytest.approx(1.0 - 0.9 * sig(16.0 * (0.0 - 0.6)), rel=1e-7)
    # training targets of the visibility cache are V in every channel
    P = 50
    pts = wl.make_points(24, P)
    idx, d, t = oracle.train_batch(pts, packed, 200, 3, 0, 0, output=oracle.OUTPUT_VISIBILITY)
    vv = oracle.visibility(packed, pts, idx, d)
    np.testing.assert_array_equal(t, np.repeat(vv[:, None], 3, 1))
    assert (vv >= 0.1).all() and (vv <= 1.0).all()
    # a radiance cache on the occluded scene learns V L
    _, _, t2 = oracle.train_batch(pts, packed, 200, 3, 0, 0, output=oracle.OUTPUT_RADIANCE_OCCLUDED)
    np.testing.assert_array_equal(t2, vv[:, None] * oracle.field(packed, pts, idx, d))


def test_visibility_cache_special_cases():
    P, N, W = 40, 8, 64
    pts = wl.make_points(25, P)
    lobes = wl.make_lobes(25).packed()
    w = wl.make_weights(25, W).copy()
    dirs = oracle.sample_dirs(pts, N, 4, 1)
    idx = np.repeat(np.arange(P), N + 1)
    L = oracle.field(lobes, pts, idx, dirs.reshape(-1, 3)).reshape(P, N + 1, 3)
    V = oracle.visibility(lobes, pts, idx, dirs.reshape(-1, 3)).reshape(P, N + 1)
    # zero output layer: sigmoid(0) = 1/2, so F_c is half the mean radiance of the cache directions
    w0 = w.copy()
    w0[-3 * W:] = 0.0
    _, c, r = oracle.estimate(pts, lobes, w0, W, N, 4, 1, output=oracle.OUTPUT_VISIBILITY)
    np.testing.assert_allclose(c, 0.5 * L[:, :N].mean(1), rtol=1e-13)
    np.testing.assert_allclose(r, (V[:, N, None] - 0.5) * L[:, N], rtol=1e-12, atol=1e-15)
    # the exact integrand in place of the network: no residual, F_c the mean of V L
    tl, c, r = oracle.estimate(pts, lobes, None, W, N, 4, 1, plug_in=True, output=oracle.OUTPUT_VISIBILITY)
    assert np.abs(r).max() == 0.0
    np.testing.assert_allclose(c, (V[:, :N, None] * L[:, :N]).mean(1), rtol=1e-13)
    # a radiance cache on the occluded scene: exp outputs, residual sample V L, F_c unchanged
    tl2, c2, r2 = oracle.estimate(pts, lobes, w, W, N, 4, 1, output=oracle.OUTPUT_RADIANCE_OCCLUDED)
    _, c0, r0 = oracle.estimate(pts, lobes, w, W, N, 4, 1)
    np.testing.assert_array_equal(c2, c0)
    np.testing.assert_allclose(r2 - r0, (V[:, N, None] - 1.0) * L[:, N], rtol=1e-12, atol=1e-15)
    # the network's visibility prediction is a sigmoid of the radiance cache's log-output
    y_rad = oracle.infer(pts, idx, dirs.reshape(-1, 3), w, W)
    y_vis = oracle.infer(pts, idx, dirs.reshape(-1, 3), w, W, output=oracle.OUTPUT_VISIBILITY)
    np.testing.assert_allclose(y_vis, y_rad / (1.0 + y_rad), rtol=1e-13)


def test_visibility_cache_estimator_unbiased():
    # mean over seeds of the two-level estimate with the visibility cache (random weights)
    # against the quadrature of V L: aggregate z over points and channels
    P, N, S, W = 24, 4, 600, 64
    pts = wl.make_points(26, P)
    lobes = wl.make_lobes(26).packed()
    w = wl.make_weights(26, W)
    F = oracle.quadrature(pts, lobes, oracle.OUTPUT_VISIBILITY, 256)
    est = np.stack([oracle.estimate(pts, lobes, w, W, N, 1000 + s, 0, output=oracle.OUTPUT_VISIBILITY)[0]
                    for s in range(S)])
    mean, var = est.mean(0), est.var(0, ddof=1)
    Z = (mean - F).sum() / math.sqrt((var / S).sum())
    assert abs(Z) < 4.5, Z


def test_visibility_cache_gradient_finite_differences():
    width, B = 64, 6
    pts = wl.make_points(27, 32)
    lobes = wl.make_lobes(27).packed()
    w = wl.make_weights(27, width).astype(np.float64)
    idx, dirs, target = oracle.train_batch(pts, lobes, B, 9, 0, 0, output=oracle.OUTPUT_VISIBILITY)
    vis = oracle.OUTPUT_VISIBILITY
    loss, g = oracle.loss_grad(pts, idx, dirs, target, w, width, output=vis)
    feat = npref.encode(npref.inputs_of(pts, idx, dirs))
    y0, pre0 = npref.forward(feat, w, width)
    s0 = y0 / (1.0 + y0)              # sigmoid(z) = e^z / (1 + e^z)
    den = s0 ** 2 + 1e-2
    assert loss == pytest.approx(((s0 - target) ** 2 / den).sum() / (3 * B), rel=1e-12)
    rng = np.random.default_rng(2)
    n = w.shape[0]
    check = np.concatenate([rng.choice(n, 150, replace=False), np.arange(n - 3 * width, n - 3 * width + 20)])
    h = 1e-4
    used = 0
    for i in check:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        yp, prep = npref.forward(feat, wp, width)
        ym, prem = npref.forward(feat, wm, width)
        if any(np.any((a > 0) != (b > 0)) or np.any((a > 0) != (c > 0)) for a, b, c in zip(pre0, prep, prem)):
            continue
        sp, sm_ = yp / (1 + yp), ym / (1 + ym)
        lp = ((sp - target) ** 2 / den).sum() / (3 * B)   # denominator held at w (stop-gradient)
        lm = ((sm_ - target) ** 2 / den).sum() / (3 * B)
        fd = (lp - lm) / (2 * h)
        scale = max(abs(fd), 1e-6 * np.abs(g).max())
        assert abs(fd - g[i]) <= 1e-6 * scale + 1e-11, (i, fd, g[i])
        used += 1
    assert used > 140


# ------------------------------------------------------------------------------------------
# Biased estimator with the balanced termination heuristic (Sec. "Path Termination Heuristics")

@pytest.mark.parametrize("N", [1, 4, 16])
def test_bth_continuation_fraction_closed_form(N):
    # cos(theta) of a cosine-weighted direction has density 2c on [0, 1], so the expected
    # continuation probability is int_0^1 c / (c + N) 2c dc = 2 (1/2 - N + N^2 ln((N + 1) / N))
    P = 200_000
    pts = wl.make_points(21, P)
    lobes = wl.make_lobes(21).packed()
    w = wl.make_weights(21, 64)
    _, cont = oracle.estimate_biased(pts, lobes, w, 64, N, 3, 0)
    expect = 2.0 * (0.5 - N + N * N * math.log((N + 1.0) / N))
    sd = math.sqrt(expect * (1 - expect) / P)
    assert abs(cont.mean() - expect) < 5 * sd, (cont.mean(), expect)


def test_bth_decision_and_outputs():
    # the squared-form decision equals the paper's xi > P_s with P_s = p / (p + N / pi),
    # p = cos / pi, where xi is not within rounding of P_s; stopped points carry F_c, continued
    # points the field (or the given radiance) along the scattering direction
    P, N, seed, frame = 20_000, 4, 9, 2
    pts = wl.make_points(22, P)
    lobes = wl.make_lobes(22).packed()
    w = wl.make_weights(22, 64)
    out, cont = oracle.estimate_biased(pts, lobes, w, 64, N, seed, frame)
    _, fc, _ = oracle.estimate(pts, lobes, w, 64, N, seed, frame)
    dirs = oracle.sample_dirs(pts, N, seed, frame)[:, N, :]
    n = np.stack([pts.nx, pts.ny, pts.nz], 1).astype(np.float64)
    cos = (n * dirs).sum(1)
    p_s = (cos / np.pi) / (cos / np.pi + N / np.pi)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    X = [int(oracle.philox([p >> 2, 0, frame, 6], key)[p & 3]) >> 8 for p in range(P)]
    xi = np.array(X) * 2.0 ** -24
    clear = np.abs(xi - p_s) > 1e-9
    assert clear.sum() > P - 5
    np.testing.assert_array_equal(cont[clear] == 0, (xi > p_s)[clear])
    # every decision, near-ties included, against xi > P_s evaluated in 60-digit decimal
    # arithmetic from the exact 24-bit uniforms (u1 of the residual direction: counter
    # (p >> 1, 0, frame, 4), word 0 or 2 by p & 1)
    with decimal.localcontext() as ctx:
        ctx.prec = 60
        for p in range(P):
            U = int(oracle.philox([p >> 1, 0, frame, 4], key)[2 * (p & 1)]) >> 8
            c = (1 - decimal.Decimal(U) / 2 ** 24).sqrt()
            assert (cont[p] == 0) == (decimal.Decimal(X[p]) / 2 ** 24 > c / (c + N)), p
    stop = cont == 0
    np.testing.assert_array_equal(out[stop], fc[stop])
    np.testing.assert_array_equal(out[~stop], oracle.field(lobes, pts, None, dirs)[~stop])
    assert 0 < (~stop).sum() < P
    R = np.random.default_rng(0).uniform(0, 1, (P, 3))
    out2, cont2 = oracle.estimate_biased(pts, lobes, w, 64, N, seed, frame, rrad=R)
    np.testing.assert_array_equal(cont2, cont)
    np.testing.assert_array_equal(out2[~stop], R[~stop])
    np.testing.assert_array_equal(out2[stop], fc[stop])


# ------------------------------------------------------------------------------------------
# Loss variants of Sec. "Radiance Cache Optimization": plain L2 and the residual-variance loss

@pytest.mark.parametrize("kind", [oracle.LOSS_L2, oracle.LOSS_VAR])
def test_loss_variants_value_and_finite_differences(kind):
    # the loss value against a numpy forward pass, and the gradient against central finite
    # differences of the loss itself (for the variance loss the batch estimate of F_r moves with
    # the weights too: its derivative must add nothing)
    width, B = 64, 6
    pts = wl.make_points(19, 32)
    lobes = wl.make_lobes(19).packed()
    w = wl.make_weights(19, width).astype(np.float64)
    idx, dirs, target = oracle.train_batch(pts, lobes, B, 7, 0, 0)
    loss, g = oracle.loss_grad(pts, idx, dirs, target, w, width, kind=kind)
    feat = npref.encode(npref.inputs_of(pts, idx, dirs))
    y0, pre0 = npref.forward(feat, w, width)
    d = y0 - target
    if kind == oracle.LOSS_VAR:
        d = d + (target - y0).mean(axis=0)
    assert loss == pytest.approx((d ** 2).sum() / (3 * B), rel=1e-12)
    rng = np.random.default_rng(1)
    n = w.shape[0]
    check = np.concatenate([rng.choice(n, 200, replace=False), np.arange(n - 3 * width, n - 3 * width + 20)])
    h = 1e-4
    used = 0
    for i in check:
        wp = w.copy(); wp[i] += h
        wm = w.copy(); wm[i] -= h
        _, prep = npref.forward(feat, wp, width)
        _, prem = npref.forward(feat, wm, width)
        if any(np.any((a > 0) != (b > 0)) or np.any((a > 0) != (c > 0)) for a, b, c in zip(pre0, prep, prem)):
            continue
        lp, _ = oracle.loss_grad(pts, idx, dirs, target, wp, width, kind=kind, want_grad=False)
        lm, _ = oracle.loss_grad(pts, idx, dirs, target, wm, width, kind=kind, want_grad=False)
        fd = (lp - lm) / (2 * h)
        scale = max(abs(fd), 1e-6 * np.abs(g).max())
        assert abs(fd - g[i]) <= 1e-6 * scale + 1e-11, (i, fd, g[i])
        used += 1
    assert used > 180


def test_loss_variant_special_cases():
    width, B = 64, 40
    pts = wl.make_points(20, 64)
    lobes = wl.make_lobes(20).packed()
    w = wl.make_weights(20, width).astype(np.float64)
    idx, dirs, target = oracle.train_batch(pts, lobes, B, 8, 0, 0)
    y = oracle.infer(pts, idx, dirs, w, width)
    shift = np.array([0.3, -0.2, 1.1])
    # the variance loss only sees the targets up to a constant per channel
    la, ga = oracle.loss_grad(pts, idx, dirs, target, w, width, kind=oracle.LOSS_VAR)
    lb, gb = oracle.loss_grad(pts, idx, dirs, target + shift, w, width, kind=oracle.LOSS_VAR)
    assert lb == pytest.approx(la, rel=1e-10)
    assert np.linalg.norm(gb - ga) <= 1e-9 * np.linalg.norm(ga)
    # targets equal to the cache's own predictions (plus a constant for the variance loss): zero
    for kind, t in ((oracle.LOSS_L2, y), (oracle.LOSS_VAR, y + shift), (oracle.LOSS_REL_L2, y)):
        l0, g0 = oracle.loss_grad(pts, idx, dirs, t, w, width, kind=kind)
        assert abs(l0) <= 1e-24 and np.abs(g0).max() <= 1e-12
    # the relative loss with a huge epsilon is the plain L2 loss divided by epsilon
    big = 1e12
    lr, gr = oracle.loss_grad(pts, idx, dirs, target, w, width, eps=big, kind=oracle.LOSS_REL_L2)
    l2, g2 = oracle.loss_grad(pts, idx, dirs, target, w, width, kind=oracle.LOSS_L2)
    assert lr * big == pytest.approx(l2, rel=1e-9)
    assert np.linalg.norm(gr * big - g2) <= 1e-9 * np.linalg.norm(g2)


# ------------------------------------------------------------------------------------------
# Adam closed forms

def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    n = 1000
    w0 = rng.normal(size=n)
    g = rng.normal(size=n) * 10.0 ** rng.uniform(-6, 2, size=n)
    w = w0.copy(); m = np.zeros(n); v = np.zeros(n)
    oracle.adam(w, m, v, g, 1, lr=1e-3)
    np.testing.assert_allclose(w - w0, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-18)


def test_adam_constant_gradient_bias_correction():
    # with a constant gradient the bias-corrected moments are exactly g and g^2 at every step
    rng = np.random.default_rng(2)
    n = 100
    g = rng.normal(size=n)
    w = np.zeros(n); m = np.zeros(n); v = np.zeros(n)
    prev = w.copy()
    for t in range(1, 30):
        oracle.adam(w, m, v, g, t, lr=1e-2)
        np.testing.assert_allclose(w - prev, -1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        prev = w.copy()


# ------------------------------------------------------------------------------------------
# Training samples

def test_train_batch_ranges_and_uniform_points():
    P = 50
    pts = wl.make_points(19, P)
    lobes = wl.make_lobes(19).packed()
    B = 20000
    idx, d, t = oracle.train_batch(pts, lobes, B, 3, 4, 2)
    assert idx.min() >= 0 and idx.max() < P
    counts = np.bincount(idx, minlength=P)
    chi2 = ((counts - B / P) ** 2 / (B / P)).sum()
    assert chi2 < scipy.stats.chi2.ppf(0.9999, P - 1)
    nrm = np.stack([pts.nx[idx], pts.ny[idx], pts.nz[idx]], axis=1).astype(np.float64)
    assert np.all(np.einsum("bd,bd->b", d, nrm) >= 0)
    np.testing.assert_allclose(t, oracle.field(lobes, pts, idx, d), rtol=1e-15)
    # point index = floor(r0 * P / 2^32) of Philox(ctr=(b, step, frame, 5))
    key = [3, 0]
    for b in (0, 1, 777):
        r = oracle.philox([b, 2, 4, 5], key)
        assert idx[b] == (int(r[0]) * P) >> 32
