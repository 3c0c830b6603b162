"""FP64 CPU oracle for the NIRC two-level Monte Carlo hot path.

TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The HIP library and its Python binding never do; the two share no code.

Thin ctypes wrapper over ``nirc_oracle.c`` (plain C, double precision).  Every function takes
numpy arrays; inputs come from the seeded workload generator, never from the HIP path.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_f32p = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_int = ctypes.c_int
_dbl = ctypes.c_double


class _Opt:
    """ndpointer that also accepts None (NULL)."""

    def __init__(self, base):
        self.base = base

    def from_param(self, obj):
        if obj is None:
            return None
        return self.base.from_param(obj)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = ctypes.CDLL(path)
        L.oracle_philox.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_philox.restype = None
        L.oracle_sample_dirs.argtypes = [_i64, _f32p, _f32p, _f32p, _Opt(_i64p), _int, _u64, _u64, _f64p]
        L.oracle_encode.argtypes = [_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p]
        L.oracle_infer.argtypes = [_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p, _int, _int, _f64p]
        L.oracle_visibility.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _Opt(_i32p), _f64p, _f64p]
        L.oracle_quadrature.argtypes = [_i64] + [_f32p] * 6 + [_f32p, _int, _int, _f64p]
        L.oracle_field.argtypes = [_i64, _f32p, _f32p, _f32p, _f32p, _Opt(_i32p), _f64p, _f64p]
        L.oracle_estimate.argtypes = ([_i64] + [_f32p] * 7 + [_f32p, _f64p, _int, _int, _int, _u64, _u64,
                                      _Opt(_f64p), _int, _Opt(_f64p), _Opt(_f64p), _Opt(_f64p)])
        L.oracle_estimate_biased.argtypes = ([_i64] + [_f32p] * 7 + [_f32p, _f64p, _int, _int, _int, _u64, _u64,
                                             _Opt(_f64p), _f64p, _Opt(_i32p)])
        L.oracle_bessel_i0.argtypes = [_dbl]
        L.oracle_bessel_i0.restype = _dbl
        L.oracle_gauss_legendre.argtypes = [_int, _f64p, _f64p]
        L.oracle_J.argtypes = [_dbl, _dbl, _int]
        L.oracle_J.restype = _dbl
        L.oracle_closed_form.argtypes = [_i64] + [_f32p] * 6 + [_f32p, _int, _f64p]
        L.oracle_second_moment.argtypes = [_i64] + [_f32p] * 6 + [_f32p, _int, _f64p]
        L.oracle_loss_grad.argtypes = ([_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p, _f64p, _int, _int,
                                       _dbl, _int, _int, _Opt(_f64p)])
        L.oracle_loss_grad.restype = _dbl
        L.oracle_adam.argtypes = [_i64, _f64p, _f64p, _f64p, _f64p, _i64, _dbl, _dbl, _dbl, _dbl]
        L.oracle_train_batch.argtypes = ([_i64] + [_f32p] * 6 + [_f32p, _i64, _u64, _u64, ctypes.c_uint32, _int,
                                         _i32p, _f64p, _f64p])
        L.oracle_n_params.argtypes = [_int]
        L.oracle_n_params.restype = _i64
        L.oracle_threads.argtypes = []
        L.oracle_threads.restype = _int
        L.oracle_set_threads.argtypes = [_int]
        L.oracle_set_threads.restype = None
        L.oracle_hash_entries.argtypes = [_int, _int, _dbl]
        L.oracle_hash_entries.restype = _i64
        L.oracle_hash_n_params.argtypes = [_int, _int, _int, _dbl]
        L.oracle_hash_n_params.restype = _i64
        L.oracle_hash_levels.argtypes = [_int, _int, _dbl, _i64p, _i64p, _i32p]
        L.oracle_sh.argtypes = [_i64, _f64p, _f64p]
        L.oracle_hash_encode.argtypes = ([_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p, _int, _int, _dbl,
                                         _f64p])
        L.oracle_hash_infer.argtypes = ([_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p, _int, _int, _int, _dbl,
                                        _f64p])
        L.oracle_hash_estimate.argtypes = ([_i64] + [_f32p] * 7 + [_f32p, _f64p, _int, _int, _int, _dbl, _int, _u64,
                                           _u64, _Opt(_f64p), _Opt(_f64p), _Opt(_f64p), _Opt(_f64p),
                                           _Opt(_f64p)])
        L.oracle_hash_loss_grad.argtypes = ([_i64] + [_f32p] * 7 + [_Opt(_i32p), _f64p, _f64p, _f64p, _int, _int,
                                            _int, _dbl, _dbl, _int, _int, _Opt(_f64p)])
        L.oracle_hash_loss_grad.restype = _dbl
        _lib = L
    return _lib


def _pts(points):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in points.arrays()]


def _w64(w):
    return np.ascontiguousarray(w, dtype=np.float64)


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def set_threads(n: int) -> None:
    """Set the OpenMP thread count of the oracle's parallel loops (timing only)."""
    lib().oracle_set_threads(int(n))


def n_params(width: int) -> int:
    return int(lib().oracle_n_params(width))


def philox(ctr, key):
    out = np.zeros(4, np.uint32)
    lib().oracle_philox(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def sample_dirs(points, n_cache: int, seed: int, frame: int, ids=None) -> np.ndarray:
    """[P, n_cache+1, 3] FP64 directions; the last one of each point is the residual direction.
    ids: for a subset of a frame's points, the frame index of each (its Philox counter)."""
    P = points.count
    out = np.zeros((P, n_cache + 1, 3), np.float64)
    i64 = None if ids is None else np.ascontiguousarray(ids, np.int64)
    assert i64 is None or i64.shape == (P,)
    lib().oracle_sample_dirs(P, points.nx, points.ny, points.nz, i64, n_cache, seed, frame, out)
    return out


def encode(points, point_idx, dirs) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros((Q, 160), np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    lib().oracle_encode(Q, *_pts(points), idx, dirs, out)
    return out


OUTPUT_RADIANCE, OUTPUT_VISIBILITY, OUTPUT_RADIANCE_OCCLUDED = 0, 1, 2


def infer(points, point_idx, dirs, w, width: int, output: int = OUTPUT_RADIANCE) -> np.ndarray:
    """Cache predictions for explicit queries (the visibility for output 1)."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros((Q, 3), np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    lib().oracle_infer(Q, *_pts(points), idx, dirs, _w64(w), width, int(output), out)
    return out


def visibility(lobes_packed, points, point_idx, dirs) -> np.ndarray:
    """The synthetic visibility V(x, w) of the visibility-cache workload, [Q] FP64."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros(Q, np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    p = _pts(points)
    lib().oracle_visibility(Q, np.ascontiguousarray(lobes_packed, np.float32), p[0], p[1], p[2], idx, dirs, out)
    return out


def quadrature(points, lobes_packed, output: int = OUTPUT_RADIANCE, n_nodes: int = 256) -> np.ndarray:
    """F = (1/pi) int V L cos over the hemisphere by tensor Gauss-Legendre quadrature, [P, 3]."""
    P = points.count
    out = np.zeros((P, 3), np.float64)
    p = _pts(points)
    lib().oracle_quadrature(P, p[0], p[1], p[2], p[3], p[4], p[5], np.ascontiguousarray(lobes_packed, np.float32),
                            int(output), n_nodes, out)
    return out


def field(lobes_packed, points, point_idx, dirs) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros((Q, 3), np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    p = _pts(points)
    lib().oracle_field(Q, np.ascontiguousarray(lobes_packed, np.float32), p[0], p[1], p[2], idx, dirs, out)
    return out


def estimate(points, lobes_packed, w, width: int, n_cache: int, seed: int, frame: int,
             dirs=None, plug_in: bool = False, output: int = OUTPUT_RADIANCE):
    """Two-level estimator per point: returns (F_tl, F_c, F_r), each [P, 3] FP64."""
    P = points.count
    tl = np.zeros((P, 3), np.float64)
    c = np.zeros((P, 3), np.float64)
    r = np.zeros((P, 3), np.float64)
    d = None if dirs is None else np.ascontiguousarray(dirs, np.float64).reshape(P * (n_cache + 1) * 3)
    wd = _w64(w) if w is not None else np.zeros(n_params(width), np.float64)
    lib().oracle_estimate(P, *_pts(points), np.ascontiguousarray(lobes_packed, np.float32), wd, width, int(output),
                          n_cache, seed, frame, d, int(plug_in), tl, c, r)
    return tl, c, r


def estimate_biased(points, lobes_packed, w, width: int, n_cache: int, seed: int, frame: int, rrad=None,
                    output: int = OUTPUT_RADIANCE):
    """Biased estimate with the balanced termination heuristic at the shading point: (out [P,3],
    continued [P] int32)."""
    P = points.count
    out = np.zeros((P, 3), np.float64)
    cont = np.zeros(P, np.int32)
    rr = None if rrad is None else np.ascontiguousarray(rrad, np.float64).reshape(P, 3)
    lib().oracle_estimate_biased(P, *_pts(points), np.ascontiguousarray(lobes_packed, np.float32), _w64(w), width,
                                 int(output), n_cache, seed, frame, rr, out, cont)
    return out, cont


def bessel_i0(z: float) -> float:
    return float(lib().oracle_bessel_i0(z))


def gauss_legendre(n: int):
    x = np.zeros(n, np.float64)
    w = np.zeros(n, np.float64)
    lib().oracle_gauss_legendre(n, x, w)
    return x, w


def J(kappa: float, t: float, n_nodes: int = 256) -> float:
    return float(lib().oracle_J(kappa, t, n_nodes))


def closed_form(points, lobes_packed, n_nodes: int = 256) -> np.ndarray:
    """F(x, n) = (1/pi) * cosine-weighted hemispherical integral of the field, [P, 3] FP64."""
    P = points.count
    out = np.zeros((P, 3), np.float64)
    p = _pts(points)
    lib().oracle_closed_form(P, p[0], p[1], p[2], p[3], p[4], p[5],
                             np.ascontiguousarray(lobes_packed, np.float32), n_nodes, out)
    return out


def second_moment(points, lobes_packed, n_nodes: int = 256) -> np.ndarray:
    """E[L^2] under cosine-weighted sampling per point and channel, [P, 3] FP64."""
    P = points.count
    out = np.zeros((P, 3), np.float64)
    p = _pts(points)
    lib().oracle_second_moment(P, p[0], p[1], p[2], p[3], p[4], p[5],
                               np.ascontiguousarray(lobes_packed, np.float32), n_nodes, out)
    return out


LOSS_REL_L2, LOSS_L2, LOSS_VAR = 0, 1, 2


def loss_grad(points, point_idx, dirs, target, w, width: int, eps: float = 1e-2, frozen: bool = True,
              want_grad: bool = True, kind: int = LOSS_REL_L2, output: int = 0):
    """Training loss (kind: relative L2, plain L2 or the residual-variance loss) and its weight
    gradient (FP64)."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    B = dirs.shape[0]
    g = np.zeros(n_params(width), np.float64) if want_grad else None
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    loss = lib().oracle_loss_grad(B, *_pts(points), idx, dirs, np.ascontiguousarray(target, np.float64).reshape(-1),
                                  _w64(w), width, int(output), eps, int(frozen), int(kind), g)
    return float(loss), g


def adam(w, m, v, g, t: int, lr: float = 1e-3, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step in place on FP64 arrays (t = 1 for the first step)."""
    lib().oracle_adam(w.shape[0], w, m, v, np.ascontiguousarray(g, np.float64), t, lr, b1, b2, eps)


def train_batch(points, lobes_packed, B: int, seed: int, frame: int, step: int, output: int = 0):
    """Training samples of one step: (point index [B] int32, directions [B,3], targets [B,3])."""
    idx = np.zeros(B, np.int32)
    d = np.zeros((B, 3), np.float64)
    t = np.zeros((B, 3), np.float64)
    p = _pts(points)
    lib().oracle_train_batch(points.count, p[0], p[1], p[2], p[3], p[4], p[5],
                             np.ascontiguousarray(lobes_packed, np.float32), B, seed, frame, step, int(output), idx, d,
                             t)
    return idx, d, t


def mrse(estimate_rgb, reference_rgb, eps: float = 1e-2) -> float:
    """Mean relative squared error over points and channels: mean((F_hat - F)^2 / (F^2 + eps))."""
    e = np.asarray(estimate_rgb, np.float64)
    r = np.asarray(reference_rgb, np.float64)
    return float(np.mean((e - r) ** 2 / (r * r + eps)))


# ------------------------------------------------------------------------------------------
# The paper's own cache input: hash grid on x, spherical harmonics of w, identity / one-blob
# surface values (64 inputs).  `grid` is (log2_table, base_res, growth).

HASH_GRID = (18, 16, 1.5)


def hash_entries(grid=HASH_GRID) -> int:
    return int(lib().oracle_hash_entries(int(grid[0]), int(grid[1]), float(grid[2])))


def hash_n_params(width: int, grid=HASH_GRID) -> int:
    return int(lib().oracle_hash_n_params(width, int(grid[0]), int(grid[1]), float(grid[2])))


def hash_mlp_params(width: int) -> int:
    return width * 64 + 3 * width * width + 3 * width


def hash_levels(grid=HASH_GRID):
    """(resolution [12], first entry [12], dense flag [12]) of the hash grid's levels."""
    res = np.zeros(12, np.int64)
    off = np.zeros(12, np.int64)
    dense = np.zeros(12, np.int32)
    lib().oracle_hash_levels(int(grid[0]), int(grid[1]), float(grid[2]), res, off, dense)
    return res, off, dense


def sh(dirs) -> np.ndarray:
    """Real spherical harmonics of degree <= 4, [Q, 25] FP64 (index l^2 + l + m)."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    out = np.zeros((dirs.shape[0], 25), np.float64)
    lib().oracle_sh(dirs.shape[0], dirs, out)
    return out


def hash_encode(points, point_idx, dirs, table, grid=HASH_GRID) -> np.ndarray:
    """The 64 inputs of each query, [Q, 64] FP64 (table: [entries * 2])."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros((Q, 64), np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    lib().oracle_hash_encode(Q, *_pts(points), idx, dirs, _w64(table), int(grid[0]), int(grid[1]),
                             float(grid[2]), out)
    return out


def hash_infer(points, point_idx, dirs, w, width: int = 64, grid=HASH_GRID) -> np.ndarray:
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    Q = dirs.shape[0]
    out = np.zeros((Q, 3), np.float64)
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    lib().oracle_hash_infer(Q, *_pts(points), idx, dirs, _w64(w), width, int(grid[0]), int(grid[1]),
                            float(grid[2]), out)
    return out


def hash_estimate(points, lobes_packed, w, n_cache: int, seed: int, frame: int, width: int = 64,
                  grid=HASH_GRID, dirs=None, rrad=None):
    """Two-level estimator of the hash-input cache: (F_tl, F_c, F_r), each [P, 3] FP64."""
    P = points.count
    tl = np.zeros((P, 3), np.float64)
    c = np.zeros((P, 3), np.float64)
    r = np.zeros((P, 3), np.float64)
    d = None if dirs is None else np.ascontiguousarray(dirs, np.float64).reshape(P * (n_cache + 1) * 3)
    rr = None if rrad is None else np.ascontiguousarray(rrad, np.float64).reshape(P * 3)
    lib().oracle_hash_estimate(P, *_pts(points), np.ascontiguousarray(lobes_packed, np.float32), _w64(w), width,
                               int(grid[0]), int(grid[1]), float(grid[2]), n_cache, seed, frame, d, rr, tl, c, r)
    return tl, c, r


def hash_loss_grad(points, point_idx, dirs, target, w, width: int = 64, grid=HASH_GRID, eps: float = 1e-2,
                   frozen: bool = True, want_grad: bool = True, kind: int = LOSS_REL_L2):
    """Loss (relative L2 or L2) of the hash-input cache and its gradient over MLP and table (FP64)."""
    dirs = np.ascontiguousarray(dirs, np.float64).reshape(-1, 3)
    B = dirs.shape[0]
    g = np.zeros(hash_n_params(width, grid), np.float64) if want_grad else None
    idx = None if point_idx is None else np.ascontiguousarray(point_idx, np.int32)
    loss = lib().oracle_hash_loss_grad(B, *_pts(points), idx, dirs,
                                       np.ascontiguousarray(target, np.float64).reshape(-1), _w64(w), width,
                                       int(grid[0]), int(grid[1]), float(grid[2]), eps, int(frozen), int(kind), g)
    return float(loss), g

