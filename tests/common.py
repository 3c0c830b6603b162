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
        self.idx = np.ascontiguousarray(self.idx[keep])
        self.d32 = np.ascontiguousarray(self.d32[keep])
        self.t32 = np.ascontiguousarray(self.t32[keep])
        return int((~keep).sum())


def oracle_dirs32(points, n_cache, seed, frame):
    """The oracle's sampled directions of a frame rounded to FP32, [P * (n_cache + 1), 3]."""
    return np.ascontiguousarray(oracle.sample_dirs(points, n_cache, seed, frame).reshape(-1, 3), np.float32)
