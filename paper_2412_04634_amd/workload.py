"""Seeded synthetic workload: shading points, the vMF-lobe radiance field and initial MLP weights.

This module only draws inputs. It holds none of the method's arithmetic (no encoding, no network,
no estimator, no loss, no optimiser and no evaluation of the radiance field): it produces arrays
that are handed, unchanged, both to the HIP library and to the FP64 CPU oracle.

Stand-in for the paper's scenes (none of which is available): the incident radiance field is a
sum of four spherical-Gaussian (vMF-shaped) lobes whose RGB amplitudes are linear in the shading
position, and shading points are scattered uniformly in the unit cube with uniformly distributed
normals. Sizes follow the paper's evaluation setting (1920x1080 shading points, Sec. "Results",
main comparison) and its cache architecture (4 hidden layers of width 64, Sec. "Results").

Random numbers come from numpy's PCG64 seeded by a SeedSequence of (seed, stream); each kind of
input has its own stream so that, e.g., changing the point count leaves the lobes unchanged.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

N_LOBES = 4
N_INPUTS = 10          # x(3), omega(3), n(3), roughness(1)
N_FREQ = 8             # sin/cos frequencies per input
N_FEATURES = N_INPUTS * N_FREQ * 2   # 160

# generator streams
_STREAM_LOBES = 0
_STREAM_POINTS = 1
_STREAM_WEIGHTS = 2
_STREAM_HASH_TABLE = 3


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([int(seed), int(stream)])))


def _uniform_sphere(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform directions on S^2 (z = 1 - 2u, phi = 2 pi u'), FP64, shape [n, 3]."""
    u = rng.random(n)
    v = rng.random(n)
    z = 1.0 - 2.0 * u
    r = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = 2.0 * math.pi * v
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], axis=1)


@dataclasses.dataclass
class Lobes:
    """Four lobes: axis [4,3], kappa [4], alpha [4,3] and beta [4,3,3] (all FP32).

    Channel c of lobe j has amplitude alpha[j,c] + sum_d beta[j,c,d] * x_d, so amplitudes are
    linear in the shading position and non-negative on the unit cube.
    """
    axis: np.ndarray
    kappa: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray

    def packed(self) -> np.ndarray:
        """The 64-float record shared by the C ABI and the oracle: axis, kappa, alpha, beta."""
        return np.concatenate([self.axis.ravel(), self.kappa.ravel(), self.alpha.ravel(),
                               self.beta.ravel()]).astype(np.float32)

    def rotated(self, frame: int) -> "Lobes":
        """The dynamic scene: lobe axes rotate about world +z by one degree per frame."""
        ang = math.radians(float(frame))
        c, s = math.cos(ang), math.sin(ang)
        a = self.axis.astype(np.float64)
        ax = np.stack([c * a[:, 0] - s * a[:, 1], s * a[:, 0] + c * a[:, 1], a[:, 2]], axis=1)
        return Lobes(ax.astype(np.float32), self.kappa.copy(), self.alpha.copy(), self.beta.copy())


def make_lobes(seed: int) -> Lobes:
    rng = _rng(seed, _STREAM_LOBES)
    axis = _uniform_sphere(rng, N_LOBES)
    kappa = 5.0 + 45.0 * rng.random(N_LOBES)
    alpha = 0.1 + 0.9 * rng.random((N_LOBES, 3))
    beta = 0.5 * rng.random((N_LOBES, 3, 3))
    return Lobes(axis.astype(np.float32), kappa.astype(np.float32), alpha.astype(np.float32),
                 beta.astype(np.float32))


@dataclasses.dataclass
class Points:
    """Shading points as structure-of-arrays FP32: position p[3], normal n[3], roughness."""
    px: np.ndarray
    py: np.ndarray
    pz: np.ndarray
    nx: np.ndarray
    ny: np.ndarray
    nz: np.ndarray
    rough: np.ndarray

    @property
    def count(self) -> int:
        return int(self.px.shape[0])

    def arrays(self):
        return (self.px, self.py, self.pz, self.nx, self.ny, self.nz, self.rough)

    def subset(self, idx: np.ndarray) -> "Points":
        return Points(*(np.ascontiguousarray(a[idx]) for a in self.arrays()))


def make_points(seed: int, count: int) -> Points:
    rng = _rng(seed, _STREAM_POINTS)
    pos = rng.random((count, 3))
    nrm = _uniform_sphere(rng, count)
    rough = rng.random(count)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)
    return Points(f(pos[:, 0]), f(pos[:, 1]), f(pos[:, 2]), f(nrm[:, 0]), f(nrm[:, 1]),
                  f(nrm[:, 2]), f(rough))


def morton_order(points: Points, bits: int = 10) -> np.ndarray:
    """A locality order of the points: indices sorted by the Morton (Z-order) code of their
    positions quantised to 2^bits cells per axis.  Stands in for the screen-space coherence of a
    renderer's shading points when a kernel gathers by position (the set and each point's
    values are unchanged; only the order)."""
    q = [np.clip((np.asarray(a, np.float64) * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
         for a in (points.px, points.py, points.pz)]
    code = np.zeros(points.count, np.int64)
    for b in range(bits):
        for axis in range(3):
            code |= ((q[axis] >> b) & 1) << (3 * b + axis)
    return np.argsort(code, kind="stable")


def layer_shapes(width: int):
    """(rows, cols) of the five weight matrices: 160->W, 3 x (W->W), W->3 (no biases)."""
    return [(width, N_FEATURES), (width, width), (width, width), (width, width), (3, width)]


def n_params(width: int) -> int:
    return sum(r * c for r, c in layer_shapes(width))


def make_weights(seed: int, width: int) -> np.ndarray:
    """Glorot-uniform weights, row-major per layer, layers concatenated (canonical layout)."""
    rng = _rng(seed, _STREAM_WEIGHTS)
    out = []
    for rows, cols in layer_shapes(width):
        a = math.sqrt(6.0 / (rows + cols))
        out.append((a * (2.0 * rng.random((rows, cols)) - 1.0)).ravel())
    return np.concatenate(out).astype(np.float32)


HASH_INPUTS = 64      # hash grid 12 x 2, spherical harmonics 25, surface values 3 + 8 + 4


def hash_layer_shapes(width: int):
    """(rows, cols) of the five weight matrices of the hash-input cache: 64->W, 3 x (W->W), W->3."""
    return [(width, HASH_INPUTS), (width, width), (width, width), (width, width), (3, width)]


def make_hash_weights(seed: int, width: int, table_floats: int, table_scale: float = 1e-4) -> np.ndarray:
    """Glorot-uniform MLP weights (canonical layout) followed by `table_floats` trainable grid
    features drawn uniformly from [-table_scale, table_scale] (the small initial features of the
    hash-encoding literature).  The table length is the caller's: it follows from the grid."""
    rng = _rng(seed, _STREAM_WEIGHTS)
    out = []
    for rows, cols in hash_layer_shapes(width):
        a = math.sqrt(6.0 / (rows + cols))
        out.append((a * (2.0 * rng.random((rows, cols)) - 1.0)).ravel())
    trng = _rng(seed, _STREAM_HASH_TABLE)
    out.append(table_scale * (2.0 * trng.random(int(table_floats)) - 1.0))
    return np.concatenate(out).astype(np.float32)


@dataclasses.dataclass
class Scene:
    seed: int
    points: Points
    lobes: Lobes


def make_scene(seed: int, count: int) -> Scene:
    return Scene(seed, make_points(seed, count), make_lobes(seed))


# Named workloads (sizes of the paper's 1080p evaluation and of a small parity case).
WORKLOADS = {
    "tiny_64x64_n8": dict(points=64 * 64, n_cache=8, width=64, seed=1, train_batch=4096, train_steps=1),
    "1080p_n16": dict(points=1920 * 1080, n_cache=16, width=64, seed=2, train_batch=65536, train_steps=4),
}
