"""Independent numpy FP64 building blocks used only as pins for the oracle in tests.

These restate textbook operations with numpy library routines (np.sin, matrix products);
they are deliberately written differently from the oracle's loops.
"""
import numpy as np


def encode(inputs10: np.ndarray) -> np.ndarray:
    """inputs [Q,10] -> features [Q,160]: sin/cos(2^k pi v) with library sin/cos."""
    q = inputs10.shape[0]
    k = 2.0 ** np.arange(8)
    ang = np.pi * inputs10[:, :, None] * k[None, None, :]          # [Q,10,8]
    out = np.stack([np.sin(ang), np.cos(ang)], axis=-1)           # [Q,10,8,2]
    return out.reshape(q, 160)


def split_weights(w: np.ndarray, width: int):
    shapes = [(width, 160), (width, width), (width, width), (width, width), (3, width)]
    mats, off = [], 0
    for r, c in shapes:
        mats.append(np.asarray(w[off:off + r * c], np.float64).reshape(r, c))
        off += r * c
    return mats


def forward(feat: np.ndarray, w: np.ndarray, width: int):
    """Matrix chain: returns (y [Q,3], list of hidden pre-activations [Q,W])."""
    mats = split_weights(w, width)
    h = feat
    pre = []
    for l in range(4):
        z = h @ mats[l].T
        pre.append(z)
        h = np.maximum(z, 0.0)
    return np.exp(h @ mats[4].T), pre


def inputs_of(points, point_idx, dirs) -> np.ndarray:
    idx = np.arange(dirs.shape[0]) if point_idx is None else np.asarray(point_idx)
    a = points.arrays()
    cols = [a[0][idx], a[1][idx], a[2][idx], dirs[:, 0], dirs[:, 1], dirs[:, 2],
            a[3][idx], a[4][idx], a[5][idx], a[6][idx]]
    return np.stack([np.asarray(c, np.float64) for c in cols], axis=1)
