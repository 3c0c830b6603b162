"""Pins of the oracle's hash-grid / spherical-harmonics / one-blob cache input (CPU only).

Spherical harmonics: textbook closed forms of degrees 0..2, orthonormality by a quadrature that
is exact for the products involved, the addition theorem and the sign convention.  Hash grid:
partition of unity, exact reproduction of the dense levels' linear index function, the published
hash on lattice points.  One-blob: values at the bin centres.  Network: numpy matrix chain.
Gradients: central finite differences over MLP weights and table entries.  Estimator: the
zero-output special case and unbiasedness against the closed-form integral.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2412_04634_amd import workload as wl

SMALL_GRID = (10, 4, 1.5)   # T = 1024: every level from the first hashed except N_0 = 4


def _rand_dirs(n, seed):
    r = np.random.default_rng(seed)
    d = r.normal(size=(n, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def _one_point(x, n=(0.0, 0.0, 1.0), rough=0.5):
    a = [np.array([v], np.float32) for v in (*x, *n, rough)]
    return wl.Points(*a)


# ------------------------------------------------------------------------------------------
# Spherical harmonics

def test_sh_low_degrees_match_textbook_forms():
    d = _rand_dirs(200, 1)
    x, y, z = d[:, 0], d[:, 1], d[:, 2]
    Y = oracle.sh(d)
    pi = math.pi
    expect = np.stack([
        np.full_like(x, 0.5 / math.sqrt(pi)),
        math.sqrt(3 / (4 * pi)) * y, math.sqrt(3 / (4 * pi)) * z, math.sqrt(3 / (4 * pi)) * x,
        math.sqrt(15 / (4 * pi)) * x * y, math.sqrt(15 / (4 * pi)) * y * z,
        math.sqrt(5 / (16 * pi)) * (3 * z * z - 1), math.sqrt(15 / (4 * pi)) * x * z,
        math.sqrt(15 / (16 * pi)) * (x * x - y * y)], axis=1)
    np.testing.assert_allclose(Y[:, :9], expect, rtol=0, atol=1e-14)


def test_sh_orthonormal_by_exact_quadrature():
    # products of degree <= 8 polynomials: 8 Gauss-Legendre nodes in cos(theta) and 18 equispaced
    # azimuths integrate them exactly
    zn, zw = np.polynomial.legendre.leggauss(8)
    phis = 2 * np.pi * np.arange(18) / 18
    Z, PH = np.meshgrid(zn, phis, indexing="ij")
    s = np.sqrt(1 - Z * Z)
    d = np.stack([s * np.cos(PH), s * np.sin(PH), Z], axis=-1).reshape(-1, 3)
    wts = (zw[:, None] * np.full(phis.shape, 2 * np.pi / 18)[None, :]).reshape(-1)
    Y = oracle.sh(d)
    gram = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(25), atol=1e-13)


def test_sh_addition_theorem():
    Y = oracle.sh(_rand_dirs(100, 2))
    for l in range(5):
        band = Y[:, l * l:(l + 1) * (l + 1)]
        np.testing.assert_allclose((band ** 2).sum(axis=1), (2 * l + 1) / (4 * math.pi), rtol=1e-13)


def test_sh_sign_convention():
    # no Condon-Shortley phase: near the pole, cos(m phi) terms are positive at phi = 0 and
    # sin(|m| phi) terms at phi = pi / (2 |m|)
    th = 0.3
    for l in range(1, 5):
        for m in range(-l, l + 1):
            if m == 0:
                continue
            ph = 0.0 if m > 0 else math.pi / (2 * abs(m))
            d = np.array([[math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)]])
            assert oracle.sh(d)[0, l * l + l + m] > 0, (l, m)


def test_sh_is_scale_invariant_and_rotates_band_one():
    d = _rand_dirs(20, 3)
    np.testing.assert_allclose(oracle.sh(3.5 * d), oracle.sh(d), atol=1e-14)


# ------------------------------------------------------------------------------------------
# One-blob, identity values

def test_oneblob_bin_centres_and_identity_slots():
    for i in range(8):
        pts = _one_point((0.2, 0.4, 0.6), n=(0.6, 0.0, 0.8), rough=(i + 0.5) / 8)
        table = np.zeros(2 * oracle.hash_entries(SMALL_GRID))
        e = oracle.hash_encode(pts, None, np.array([[0.0, 0.0, 1.0]]), table, SMALL_GRID)[0]
        blob = e[52:60]
        assert blob[i] == pytest.approx(1.0, abs=float(np.spacing(np.float32(1.0))))
        for j in range(8):
            r = np.float64(np.float32((i + 0.5) / 8))
            assert blob[j] == pytest.approx(math.exp(-0.5 * (8 * (r - (j + 0.5) / 8)) ** 2), rel=1e-12)
        np.testing.assert_allclose(e[49:52], np.float32([0.6, 0.0, 0.8]), rtol=0)
        assert list(e[60:64]) == [1.0, 1.0, 1.0, 0.0]


# ------------------------------------------------------------------------------------------
# Hash grid

def test_grid_levels_follow_the_resolution_rule():
    res, off, dense = oracle.hash_levels()
    expect = [math.floor(16 * 1.5 ** l) for l in range(12)]
    assert list(res) == expect
    T = 1 << 18
    sizes = [(r + 1) ** 3 if (r + 1) ** 3 <= T else T for r in expect]
    assert list(off) == list(np.concatenate([[0], np.cumsum(sizes)[:-1]]))
    assert list(dense) == [int((r + 1) ** 3 <= T) for r in expect]
    assert oracle.hash_entries() == sum(sizes)


def test_grid_partition_of_unity():
    pts = wl.make_points(3, 50)
    table = np.full(2 * oracle.hash_entries(), 0.75)
    e = oracle.hash_encode(pts, None, _rand_dirs(50, 4), table)
    np.testing.assert_allclose(e[:, :24], 0.75, rtol=1e-14)


def test_dense_levels_reproduce_their_linear_index():
    # with table value = entry index (feature 0) on a dense level, trilinear interpolation returns
    # the (linear) index function at the scaled position: p0 + (N+1) p1 + (N+1)^2 p2
    res, off, dense = oracle.hash_levels()
    n = oracle.hash_entries()
    table = np.zeros(2 * n)
    table[0::2] = np.arange(n, dtype=np.float64)
    pts = wl.make_points(5, 64)
    e = oracle.hash_encode(pts, None, _rand_dirs(64, 5), table)
    x = np.stack([pts.px, pts.py, pts.pz], axis=1).astype(np.float64)
    for l in range(12):
        if not dense[l]:
            continue
        N = res[l]
        p = x * N
        expect = off[l] + p[:, 0] + (N + 1) * p[:, 1] + (N + 1) ** 2 * p[:, 2]
        np.testing.assert_allclose(e[:, 2 * l], expect, rtol=0, atol=1e-7)


@pytest.mark.parametrize("l", [4, 7, 11])
def test_hashed_levels_use_the_published_spatial_hash(l):
    # lattice vertices of a hashed level select one entry; with value = entry index (feature 0)
    # the feature is (v0 * 1 xor v1 * 2654435761 xor v2 * 805459861) mod T (Mueller et al. 2022).
    # Positions v / N rounded to FP32 land within ~1e-7 N of the vertex, so a neighbour's entry
    # contributes at most that fraction.  Feature 1 holds 1 everywhere (partition of unity).
    res, off, dense = oracle.hash_levels()
    assert not dense[l]
    n = oracle.hash_entries()
    T = 1 << 18
    table = np.ones(2 * n)
    table[0::2] = np.arange(n, dtype=np.float64)
    N = int(res[l])
    rng = np.random.default_rng(7 + l)
    ok = 0
    for _ in range(40):
        v = rng.integers(1, N - 1, size=3)
        pts = _one_point(tuple((v / N).astype(np.float32)))
        e = oracle.hash_encode(pts, None, np.array([[0.0, 0.0, 1.0]]), table)[0]
        h = (int(v[0]) ^ ((int(v[1]) * 2654435761) & 0xFFFFFFFF) ^ ((int(v[2]) * 805459861) & 0xFFFFFFFF)) % T
        frac = np.abs(np.float32(v / N).astype(np.float64) * N - v).max()
        assert abs(e[2 * l] - (off[l] + h)) <= 3 * frac * T + 1e-9
        assert e[2 * l + 1] == pytest.approx(1.0, abs=1e-12)
        ok += 1
    assert ok == 40


# ------------------------------------------------------------------------------------------
# Network, estimator, gradient

def _hash_w(seed, grid=oracle.HASH_GRID, table_scale=1e-4):
    return wl.make_hash_weights(seed, 64, 2 * oracle.hash_entries(grid), table_scale).astype(np.float64)


def test_hash_mlp_matches_numpy_matrix_chain():
    pts = wl.make_points(8, 40)
    d = _rand_dirs(40, 8)
    w = _hash_w(8, SMALL_GRID, table_scale=0.5)
    nm = oracle.hash_mlp_params(64)
    e = oracle.hash_encode(pts, None, d, w[nm:], SMALL_GRID)
    shapes = wl.hash_layer_shapes(64)
    h, o = e, 0
    for i, (r, c) in enumerate(shapes):
        M = w[o:o + r * c].reshape(r, c)
        o += r * c
        h = h @ M.T
        if i < 4:
            h = np.maximum(h, 0.0)
    np.testing.assert_allclose(oracle.hash_infer(pts, None, d, w, 64, SMALL_GRID), np.exp(h), rtol=1e-12)


def test_hash_estimator_zero_output_layer():
    pts = wl.make_points(9, 30)
    lobes = wl.make_lobes(9).packed()
    w = _hash_w(9, SMALL_GRID)
    nm = oracle.hash_mlp_params(64)
    w[nm - 3 * 64:nm] = 0.0
    n = 6
    tl, c, r = oracle.hash_estimate(pts, lobes, w, n, 11, 2, grid=SMALL_GRID)
    assert np.all(c == 1.0)
    dirs = oracle.sample_dirs(pts, n, 11, 2)
    L = oracle.field(lobes, pts, None, dirs[:, n])
    np.testing.assert_allclose(r, L - 1.0, rtol=1e-14, atol=1e-15)
    rr = np.random.default_rng(1).random((30, 3))
    tl2, _, r2 = oracle.hash_estimate(pts, lobes, w, n, 11, 2, grid=SMALL_GRID, rrad=rr)
    np.testing.assert_allclose(r2, rr - 1.0, rtol=1e-15)


def test_hash_estimator_unbiased_over_seeds():
    P, n, S = 10, 4, 300
    pts = wl.make_points(16, P)
    lobes = wl.make_lobes(16).packed()
    w = _hash_w(16, SMALL_GRID, table_scale=0.5)
    F = oracle.closed_form(pts, lobes)
    samples = np.stack([oracle.hash_estimate(pts, lobes, w, n, 2000 + s, 0, grid=SMALL_GRID)[0]
                        for s in range(S)])
    z = (samples.mean(axis=0) - F) / (samples.std(axis=0, ddof=1) / math.sqrt(S))
    assert np.abs(z).max() < 4.5


@pytest.mark.parametrize("kind", [oracle.LOSS_REL_L2, oracle.LOSS_L2])
def test_hash_gradient_finite_differences(kind):
    B = 6
    pts = wl.make_points(21, B)
    d = _rand_dirs(B, 21)
    w = _hash_w(21, SMALL_GRID, table_scale=0.5)
    t = np.random.default_rng(21).random((B, 3)) + 0.2
    loss, g = oracle.hash_loss_grad(pts, None, d, t, w, 64, SMALL_GRID, kind=kind)
    nm = oracle.hash_mlp_params(64)
    rng = np.random.default_rng(22)
    touched = np.nonzero(g[nm:])[0] + nm
    assert touched.size > 0
    idx = np.concatenate([rng.choice(nm, 40, replace=False), rng.choice(touched, min(60, touched.size),
                                                                         replace=False)])
    h = 1e-6
    scale = np.abs(g).max()
    for i in idx:
        wp, wm = w.copy(), w.copy()
        wp[i] += h
        wm[i] -= h
        # the frozen denominator: FD of the loss whose denominator uses the unperturbed y
        fp = _frozen_loss(pts, d, t, wp, w, kind)
        fm = _frozen_loss(pts, d, t, wm, w, kind)
        assert abs((fp - fm) / (2 * h) - g[i]) <= 1e-6 * scale + 1e-7 * abs(g[i]), i
    # entries no sample touches get exactly zero
    untouched = np.setdiff1d(np.arange(nm, w.size), touched)
    assert np.all(g[untouched] == 0.0)


def _frozen_loss(pts, d, t, w, w_den, kind):
    y = oracle.hash_infer(pts, None, d, w, 64, SMALL_GRID)
    if kind == oracle.LOSS_L2:
        return float(np.mean((y - t) ** 2))
    y0 = oracle.hash_infer(pts, None, d, w_den, 64, SMALL_GRID)
    return float(np.mean((y - t) ** 2 / (y0 * y0 + 1e-2)))


def test_hash_gradient_stop_gradient_is_honoured():
    B = 4
    pts = wl.make_points(23, B)
    d = _rand_dirs(B, 23)
    w = _hash_w(23, SMALL_GRID, table_scale=0.5)
    t = np.random.default_rng(23).random((B, 3)) + 0.2
    _, g1 = oracle.hash_loss_grad(pts, None, d, t, w, 64, SMALL_GRID, frozen=True)
    _, g0 = oracle.hash_loss_grad(pts, None, d, t, w, 64, SMALL_GRID, frozen=False)
    assert np.abs(g1 - g0).max() > 1e-3 * np.abs(g1).max()


def test_hash_gradient_matches_numpy_backprop_chain():
    # the MLP part of the oracle's hash-model gradient against backpropagation written with numpy
    # matrix products on the oracle's FP64 inputs (ReLU'(0) = 0; masks from the FP64 pass)
    B = 48
    pts = wl.make_points(24, B)
    d = _rand_dirs(B, 24)
    w = _hash_w(24, SMALL_GRID, table_scale=0.5)
    t = np.random.default_rng(24).random((B, 3)) + 0.2
    nm = oracle.hash_mlp_params(64)
    e = oracle.hash_encode(pts, None, d, w[nm:], SMALL_GRID)
    mats, o = [], 0
    for r, c in wl.hash_layer_shapes(64):
        mats.append(w[o:o + r * c].reshape(r, c))
        o += r * c
    hs, masks, x = [], [], e
    for l in range(4):
        z = x @ mats[l].T
        masks.append(z > 0)
        x = np.maximum(z, 0.0)
        hs.append(x)
    y = np.exp(hs[3] @ mats[4].T)
    dz = 2 * (y - t) / (y * y + 1e-2) * y / (3 * B)
    grads = [None] * 5
    grads[4] = dz.T @ hs[3]
    delta = (dz @ mats[4]) * masks[3]
    for l in range(3, 0, -1):
        grads[l] = delta.T @ hs[l - 1]
        delta = (delta @ mats[l]) * masks[l - 1]
    grads[0] = delta.T @ e
    ref = np.concatenate([g.ravel() for g in grads])
    loss, g = oracle.hash_loss_grad(pts, None, d, t, w, 64, SMALL_GRID)
    np.testing.assert_allclose(g[:nm], ref, rtol=1e-10, atol=1e-14 * np.abs(ref).max())
    assert loss == pytest.approx(float(np.mean((y - t) ** 2 / (y * y + 1e-2))), rel=1e-12)


def test_grid_gradient_inner_product_identity():
    # sum_i T_i dL/dT_i = sum_{r, k<24} W1[r, k] dL/dW1[r, k]: both equal sum_b sum_k e_bk dL/de_bk,
    # the first through the trilinear scatter, the second through the first layer's gradient
    B = 200
    pts = wl.make_points(25, 500)
    lob = wl.make_lobes(25).packed()
    from tests.common import Samples
    sm = Samples(pts, lob, B, 26, 0, 0)
    for grid in (SMALL_GRID, oracle.HASH_GRID):
        w = _hash_w(25, grid, table_scale=0.5)
        _, g = oracle.hash_loss_grad(pts, sm.idx, sm.d, sm.t, w, 64, grid)
        nm = oracle.hash_mlp_params(64)
        W1 = w[:64 * 64].reshape(64, 64)[:, :24]
        rhs = np.sum(W1 * g[:64 * 64].reshape(64, 64)[:, :24])
        assert np.dot(w[nm:], g[nm:]) == pytest.approx(rhs, rel=1e-12)
