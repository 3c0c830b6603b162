"""ctypes binding of libnirc (include/nirc.h): argument marshalling only.

Every computation runs in the HIP library; torch provides device memory and the current
stream.  If the library is missing this module raises instead of computing anything itself.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

from . import workload

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnirc.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "nirc.h")

NIRC_FP32, NIRC_BF16, NIRC_FP16 = 0, 1, 2
NIRC_FLAG_NONFINITE_GRAD = 1
NIRC_FLAG_BAD_POINT_INDEX = 2
NIRC_LOSS_REL_L2, NIRC_LOSS_L2, NIRC_LOSS_VAR = 0, 1, 2
NIRC_OUTPUT_RADIANCE, NIRC_OUTPUT_VISIBILITY, NIRC_OUTPUT_RADIANCE_OCCLUDED = 0, 1, 2

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_sz = ctypes.c_size_t


class Config(ctypes.Structure):
    _fields_ = [("width", _i32), ("precision", _i32), ("lr", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("adam_eps", ctypes.c_float), ("loss_eps", ctypes.c_float),
                ("loss_scale", ctypes.c_float), ("loss", _i32), ("output", _i32)]


class _Points(ctypes.Structure):
    _fields_ = [("px", _vp), ("py", _vp), ("pz", _vp), ("nx", _vp), ("ny", _vp), ("nz", _vp),
                ("rough", _vp), ("count", _i64)]


class _Queries(ctypes.Structure):
    _fields_ = [("wx", _vp), ("wy", _vp), ("wz", _vp), ("point", _vp), ("count", _i64)]


class Lobes(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_float * 64)]   # axis[4][3], kappa[4], alpha[4][3], beta[4][3][3]


class _Request(ctypes.Structure):
    _fields_ = [("model", _vp), ("points", _Points), ("field", Lobes), ("n_cache", _i32), ("seed", _u64),
                ("frame", _u64), ("residual_radiance", _vp), ("out_tl", _vp), ("out_c", _vp), ("out_r", _vp)]


class _TrainRequest(ctypes.Structure):
    _fields_ = [("model", _vp), ("points", _Points), ("field", Lobes), ("batch", _i64), ("seed", _u64),
                ("frame", _u64)]


class HashGrid(ctypes.Structure):
    _fields_ = [("log2_table", _i32), ("base_res", _i32), ("growth", ctypes.c_float)]


class NircError(RuntimeError):
    pass


_lib = None


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise NircError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "nirc_n_params": (_i64, [_i32]),
            "nirc_state_bytes": (_sz, [ctypes.POINTER(Config)]),
            "nirc_workspace_bytes": (_sz, [ctypes.POINTER(Config), _i64]),
            "nirc_create": (_i32, [ctypes.POINTER(Config), _vp, _sz, _vp, _sz, _vp, _vp, ctypes.POINTER(_vp)]),
            "nirc_destroy": (_i32, [_vp]),
            "nirc_set_weights": (_i32, [_vp, _vp, _vp]),
            "nirc_get_weights": (_i32, [_vp, _vp, _vp]),
            "nirc_get_adam": (_i32, [_vp, _vp, _vp, _vp, _vp]),
            "nirc_get_state": (_i32, [_vp, _vp, _sz, _vp]),
            "nirc_set_state": (_i32, [_vp, _vp, _sz, _vp]),
            "nirc_read_flags": (_u32, [_vp, _vp]),
            "nirc_clear_flags": (_i32, [_vp, _vp]),
            "nirc_read_loss_scale": (ctypes.c_float, [_vp, _vp]),
            "nirc_encode": (_i32, [_Points, _Queries, _vp, _vp]),
            "nirc_infer": (_i32, [_vp, _Points, _Queries, _vp, _vp]),
            "tlmc_sample_dirs": (_i32, [_Points, _i32, _u64, _u64, _vp, _vp]),
            "tlmc_estimate": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i32, _u64, _u64, _vp, _vp, _vp, _vp,
                                     _vp]),
            "tlmc_estimate_biased": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i32, _u64, _u64, _vp, _vp, _vp,
                                            _vp, _vp]),
            "tlmc_reference_occluded": (_i32, [_Points, ctypes.POINTER(Lobes), _i32, _vp, _vp]),
            "tlmc_train_batch": (_i32, [_Points, ctypes.POINTER(Lobes), _i64, _u64, _u64, _u32, _i32, _vp, _vp, _vp,
                                        _vp, _vp, _vp]),
            "nirc_loss_grad": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp, _vp]),
            "nirc_backward": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp]),
            "nirc_adam_step": (_i32, [_vp, _vp, _vp]),
            "nirc_train_step": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp]),
            "nirc_train_step_static": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp]),
            "nirc_probe_mfma": (_i32, [_i32, _i32, _i32, _i32, _vp, _vp]),
            "nirc_probe_atomics": (_i32, [_i32, _i32, _i32, _vp, _i64, _vp]),
            "tlmc_reference_table": (_i32, [ctypes.POINTER(Lobes), _vp, _vp]),
            "tlmc_reference": (_i32, [_Points, ctypes.POINTER(Lobes), _vp, _vp, _vp]),
            "tlmc_frame_stats_scratch_bytes": (_sz, []),
            "tlmc_frame_stats": (_i32, [_Points, ctypes.POINTER(Lobes), _vp, _vp, _vp, _vp, ctypes.c_double, _vp,
                                        _vp, _vp]),
            "tlmc_accumulate": (_i32, [_vp, _i64, _vp, _vp, _vp]),
            "tlmc_batch_bytes": (_sz, []),
            "tlmc_batch_build": (_i32, [ctypes.POINTER(_Request), _i32, _vp]),
            "tlmc_estimate_batch": (_i32, [_vp, _i32, _i32, _i32, _vp]),
            "tlmc_unfused_workspace_bytes": (_sz, [_i64, _i32, _i32]),
            "tlmc_estimate_unfused": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i32, _u64, _u64, _i32, _vp, _sz,
                                             _vp, _vp, _vp, _vp]),
            "nirc_train_list_bytes": (_sz, []),
            "nirc_train_list_build": (_i32, [ctypes.POINTER(_TrainRequest), _i32, _i64, _vp]),
            "nirc_train_frame_batch": (_i32, [_vp, _i32, _i32, _i64, _vp]),
            "nirc_train_frame": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i64, _i32, _u64, _u64, _vp, _vp]),
            "nirc_hash_entries": (_i64, [ctypes.POINTER(HashGrid)]),
            "nirc_hash_n_params": (_i64, [ctypes.POINTER(HashGrid)]),
            "nirc_hash_levels": (_i32, [ctypes.POINTER(HashGrid), _vp, _vp, _vp]),
            "nirc_hash_state_bytes": (_sz, [ctypes.POINTER(Config), ctypes.POINTER(HashGrid)]),
            "nirc_hash_workspace_bytes": (_sz, [ctypes.POINTER(Config), ctypes.POINTER(HashGrid), _i64]),
            "nirc_hash_create": (_i32, [ctypes.POINTER(Config), ctypes.POINTER(HashGrid), _vp, _sz, _vp, _sz, _vp,
                                        _vp, ctypes.POINTER(_vp)]),
            "nirc_hash_destroy": (_i32, [_vp]),
            "nirc_hash_set_weights": (_i32, [_vp, _vp, _vp]),
            "nirc_hash_get_weights": (_i32, [_vp, _vp, _vp]),
            "nirc_hash_get_state": (_i32, [_vp, _vp, _sz, _vp]),
            "nirc_hash_set_state": (_i32, [_vp, _vp, _sz, _vp]),
            "nirc_hash_infer": (_i32, [_vp, _Points, _Queries, _vp, _vp]),
            "nirc_hash_estimate": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i32, _u64, _u64, _vp, _vp, _vp,
                                          _vp, _vp]),
            "nirc_hash_loss_grad": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp, _vp]),
            "nirc_hash_adam_step": (_i32, [_vp, _vp, _vp]),
            "nirc_hash_train_step": (_i32, [_vp, _Points, _Queries, _vp, _vp, _vp]),
            "nirc_hash_read_flags": (_u32, [_vp, _vp]),
            "nirc_hash_train_frame": (_i32, [_vp, _Points, ctypes.POINTER(Lobes), _i64, _i32, _u64, _u64, _vp, _vp]),
            "nirc_status_string": (ctypes.c_char_p, [_i32]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/nirc.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b((?:nirc|tlmc)_[a-z0-9_]+)\s*\(", text)))


def _check(status: int, what: str):
    if status != 0:
        msg = lib().nirc_status_string(status).decode()
        raise NircError(f"{what} failed: {msg} ({status})")


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(a, device):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32)).to(device)


# ------------------------------------------------------------------------------------------

class Points:
    """Shading points on the GPU (structure of arrays, FP32)."""

    def __init__(self, arrays, device="cuda"):
        self.t = [a if isinstance(a, torch.Tensor) else _dev_f32(a, device) for a in arrays]
        for a in self.t:
            assert a.dtype == torch.float32 and a.is_contiguous() and a.numel() == self.t[0].numel()
        self.count = int(self.t[0].numel())

    @classmethod
    def from_workload(cls, pts: workload.Points, device="cuda"):
        return cls(pts.arrays(), device)

    def c(self):
        return _Points(*[a.data_ptr() for a in self.t], self.count)


class Queries:
    """Cache queries: direction (SoA FP32) and point index (int32) per query."""

    def __init__(self, wx, wy, wz, point=None):
        self.wx, self.wy, self.wz = wx, wy, wz
        self.point = point
        self.count = int(wx.numel())

    @classmethod
    def from_dirs(cls, dirs: torch.Tensor, point: torch.Tensor | None = None):
        d = dirs.reshape(-1, 3)
        return cls(d[:, 0].contiguous(), d[:, 1].contiguous(), d[:, 2].contiguous(),
                   None if point is None else point.to(torch.int32).contiguous())

    def c(self):
        return _Queries(self.wx.data_ptr(), self.wy.data_ptr(), self.wz.data_ptr(),
                        None if self.point is None else self.point.data_ptr(), self.count)


def lobes_struct(packed64) -> Lobes:
    a = np.ascontiguousarray(packed64, dtype=np.float32).ravel()
    assert a.size == 64
    L = Lobes()
    ctypes.memmove(ctypes.addressof(L), a.ctypes.data, 64 * 4)
    return L


def make_config(width=64, precision=NIRC_FP32, lr=1e-3, beta1=0.9, beta2=0.999, adam_eps=1e-8,
                loss_eps=1e-2, loss_scale=1.0, loss=0, output=0) -> Config:
    """loss: NIRC_LOSS_REL_L2 (eq. 12, default), NIRC_LOSS_L2 or NIRC_LOSS_VAR.
    output: NIRC_OUTPUT_RADIANCE (default), NIRC_OUTPUT_VISIBILITY or NIRC_OUTPUT_RADIANCE_OCCLUDED."""
    return Config(width, precision, lr, beta1, beta2, adam_eps, loss_eps, loss_scale, loss, output)


def nirc_n_params(width: int) -> int:
    return int(lib().nirc_n_params(width))


def nirc_state_bytes(cfg: Config) -> int:
    return int(lib().nirc_state_bytes(ctypes.byref(cfg)))


def nirc_workspace_bytes(cfg: Config, max_batch: int) -> int:
    return int(lib().nirc_workspace_bytes(ctypes.byref(cfg), max_batch))


class Model:
    """A cache model over torch-allocated state and workspace."""

    def __init__(self, init_w, cfg: Config | None = None, max_batch: int = 65536, device="cuda",
                 workspace: torch.Tensor | None = None):
        """workspace: an existing training workspace to share (calls on the models that share it
        must not overlap); otherwise one for batches of up to max_batch is allocated."""
        self.cfg = cfg or make_config()
        self.width = self.cfg.width
        self.n_params = nirc_n_params(self.width)
        sb = nirc_state_bytes(self.cfg)
        if sb == 0:
            raise NircError("unsupported configuration")
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        if workspace is not None:
            self.workspace, wb = workspace, workspace.numel()
        else:
            wb = nirc_workspace_bytes(self.cfg, max_batch) if max_batch > 0 else 0
            self.workspace = torch.empty(max(wb, 1), dtype=torch.uint8, device=device) if wb else None
        w = init_w if isinstance(init_w, torch.Tensor) else _dev_f32(init_w, device)
        assert w.numel() == self.n_params
        self._w0 = w.contiguous()
        h = _vp()
        _check(lib().nirc_create(ctypes.byref(self.cfg), _ptr(self.state), sb, _ptr(self.workspace), wb,
                                 _ptr(self._w0), _stream(), ctypes.byref(h)), "nirc_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.nirc_destroy(h)
            self.handle = None

    def set_weights(self, w: torch.Tensor):
        self._w0 = w.contiguous()
        _check(lib().nirc_set_weights(self.handle, _ptr(self._w0), _stream()), "nirc_set_weights")

    def get_weights(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.state.device)
        _check(lib().nirc_get_weights(self.handle, _ptr(out), _stream()), "nirc_get_weights")
        return out

    def get_adam(self):
        m = torch.empty(self.n_params, dtype=torch.float32, device=self.state.device)
        v = torch.empty_like(m)
        step = torch.zeros(1, dtype=torch.int64, device=self.state.device)
        _check(lib().nirc_get_adam(self.handle, _ptr(m), _ptr(v), _ptr(step), _stream()), "nirc_get_adam")
        return m, v, step

    def get_state(self) -> torch.Tensor:
        """The whole training state as a device byte tensor (checkpoint)."""
        out = torch.empty(self.state.numel(), dtype=torch.uint8, device=self.state.device)
        _check(lib().nirc_get_state(self.handle, _ptr(out), out.numel(), _stream()), "nirc_get_state")
        return out

    def set_state(self, blob: torch.Tensor, sync: bool = True):
        """Restore a state written by get_state of a model of the same width (resume).  With
        sync=False the copy stays enqueued: blob must then be a device tensor that lives on the
        current stream until the copy has run."""
        b = blob.to(self.state.device).contiguous()
        _check(lib().nirc_set_state(self.handle, _ptr(b), b.numel(), _stream()), "nirc_set_state")
        if sync:
            torch.cuda.current_stream().synchronize()   # b may be a temporary

    def read_flags(self) -> int:
        return int(lib().nirc_read_flags(self.handle, _stream()))

    def read_loss_scale(self) -> float:
        """The current loss scale (dynamic for FP16 models); synchronises the stream."""
        return float(lib().nirc_read_loss_scale(self.handle, _stream()))

    def clear_flags(self):
        _check(lib().nirc_clear_flags(self.handle, _stream()), "nirc_clear_flags")


# ------------------------------------------------------------------------------------------
# Entry points (same names as the C ABI)

def nirc_encode(points: Points, queries: Queries) -> torch.Tensor:
    out = torch.empty((queries.count, 160), dtype=torch.float32, device=points.t[0].device)
    _check(lib().nirc_encode(points.c(), queries.c(), _ptr(out), _stream()), "nirc_encode")
    return out


def nirc_infer(model: Model, points: Points, queries: Queries) -> torch.Tensor:
    out = torch.empty((queries.count, 3), dtype=torch.float32, device=points.t[0].device)
    _check(lib().nirc_infer(model.handle, points.c(), queries.c(), _ptr(out), _stream()), "nirc_infer")
    return out


def tlmc_sample_dirs(points: Points, n_cache: int, seed: int, frame: int) -> torch.Tensor:
    out = torch.empty((points.count, n_cache + 1, 3), dtype=torch.float32, device=points.t[0].device)
    _check(lib().tlmc_sample_dirs(points.c(), n_cache, seed, frame, _ptr(out), _stream()), "tlmc_sample_dirs")
    return out


def tlmc_estimate(model: Model, points: Points, lobes, n_cache: int, seed: int, frame: int,
                  parts: bool = False, out=None, residual=None):
    """Two-level estimate per point; returns F_tl, or (F_tl, F_c, F_r) with parts=True.
    residual: the residual sample's radiance [P, 3] (FP32, on the device) at the directions
    tlmc_sample_dirs returns; None evaluates the lobe field `lobes` (which may then be None)."""
    dev = points.t[0].device
    L = None if lobes is None else (lobes if isinstance(lobes, Lobes) else lobes_struct(lobes))
    tl = out if out is not None else torch.empty((points.count, 3), dtype=torch.float32, device=dev)
    c = torch.empty_like(tl) if parts else None
    r = torch.empty_like(tl) if parts else None
    if residual is not None:
        assert residual.dtype == torch.float32 and residual.is_contiguous() and residual.numel() == 3 * points.count
    _check(lib().tlmc_estimate(model.handle, points.c(), None if L is None else ctypes.byref(L), n_cache, seed,
                               frame, _ptr(residual), _ptr(tl), _ptr(c), _ptr(r), _stream()), "tlmc_estimate")
    return (tl, c, r) if parts else tl


def tlmc_unfused_workspace_bytes(points: int, n_cache: int, stage: int) -> int:
    return int(lib().tlmc_unfused_workspace_bytes(points, n_cache, stage))


def tlmc_estimate_unfused(model: Model, points: Points, lobes, n_cache: int, seed: int, frame: int, stage: int,
                          workspace=None, parts: bool = False, out=None):
    """The estimate with the pipeline fusions undone up to `stage` (0: every query's encoded
    inputs through memory, 1: + surface encoding shared per point, 2: + direction encoding in the
    network kernel, 3: the fused estimator).  workspace: a device byte tensor of at least
    tlmc_unfused_workspace_bytes (allocated here if None)."""
    dev = points.t[0].device
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    need = tlmc_unfused_workspace_bytes(points.count, n_cache, stage)
    if workspace is None and need:
        workspace = torch.empty(need, dtype=torch.uint8, device=dev)
    tl = out if out is not None else torch.empty((points.count, 3), dtype=torch.float32, device=dev)
    c = torch.empty_like(tl) if parts else None
    r = torch.empty_like(tl) if parts else None
    _check(lib().tlmc_estimate_unfused(model.handle, points.c(), ctypes.byref(L), n_cache, seed, frame, stage,
                                       _ptr(workspace), 0 if workspace is None else workspace.numel(), _ptr(tl),
                                       _ptr(c), _ptr(r), _stream()), "tlmc_estimate_unfused")
    return (tl, c, r) if parts else tl


def tlmc_estimate_biased(model: Model, points: Points, lobes, n_cache: int, seed: int, frame: int,
                         residual=None, out=None):
    """Biased estimate with the balanced termination heuristic: (out [P,3], F_c [P,3],
    continued [P] int32)."""
    dev = points.t[0].device
    L = None if lobes is None else (lobes if isinstance(lobes, Lobes) else lobes_struct(lobes))
    b = out if out is not None else torch.empty((points.count, 3), dtype=torch.float32, device=dev)
    c = torch.empty_like(b)
    cont = torch.empty(points.count, dtype=torch.int32, device=dev)
    if residual is not None:
        assert residual.dtype == torch.float32 and residual.is_contiguous() and residual.numel() == 3 * points.count
    _check(lib().tlmc_estimate_biased(model.handle, points.c(), None if L is None else ctypes.byref(L), n_cache, seed,
                                      frame, _ptr(residual), _ptr(b), _ptr(c), _ptr(cont), _stream()),
           "tlmc_estimate_biased")
    return b, c, cont


def tlmc_train_batch(points: Points, lobes, batch: int, seed: int, frame: int, step: int, output: int = 0):
    """Training samples: (Queries with point indices, targets [B,3]); output selects the targets
    (radiance, visibility, or radiance of the occluded scene)."""
    dev = points.t[0].device
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    idx = torch.empty(batch, dtype=torch.int32, device=dev)
    wx = torch.empty(batch, dtype=torch.float32, device=dev)
    wy = torch.empty_like(wx)
    wz = torch.empty_like(wx)
    tgt = torch.empty((batch, 3), dtype=torch.float32, device=dev)
    _check(lib().tlmc_train_batch(points.c(), ctypes.byref(L), batch, seed, frame, step, output, _ptr(idx), _ptr(wx),
                                  _ptr(wy), _ptr(wz), _ptr(tgt), _stream()), "tlmc_train_batch")
    return Queries(wx, wy, wz, idx), tgt


def nirc_loss_grad(model: Model, points: Points, queries: Queries, target: torch.Tensor):
    grad = torch.empty(model.n_params, dtype=torch.float32, device=target.device)
    loss = torch.empty(1, dtype=torch.float32, device=target.device)
    _check(lib().nirc_loss_grad(model.handle, points.c(), queries.c(), _ptr(target), _ptr(grad), _ptr(loss),
                                _stream()), "nirc_loss_grad")
    return loss, grad


def nirc_backward(model: Model, points: Points, queries: Queries, d_rgb: torch.Tensor) -> torch.Tensor:
    grad = torch.empty(model.n_params, dtype=torch.float32, device=d_rgb.device)
    d = d_rgb.contiguous()
    _check(lib().nirc_backward(model.handle, points.c(), queries.c(), _ptr(d), _ptr(grad), _stream()),
           "nirc_backward")
    return grad


def nirc_adam_step(model: Model, grad: torch.Tensor):
    _check(lib().nirc_adam_step(model.handle, _ptr(grad.contiguous()), _stream()), "nirc_adam_step")


def nirc_train_step(model: Model, points: Points, queries: Queries, target: torch.Tensor, loss=None):
    _check(lib().nirc_train_step(model.handle, points.c(), queries.c(), _ptr(target), _ptr(loss), _stream()),
           "nirc_train_step")
    return loss


def nirc_probe_mfma(precision: int, iters: int, fmas: int, sink: torch.Tensor):
    """Matrix-core microbenchmark on the current stream: sink.numel() // 256 workgroups, each wave
    `iters` (a multiple of 32) iterations of 8 independent MFMAs plus `fmas` (0, 32, 64) FP32 FMAs;
    returns the FLOPs of its MFMAs (the caller times the launch)."""
    blocks = sink.numel() // 256
    _check(lib().nirc_probe_mfma(precision, iters, fmas, blocks, _ptr(sink), _stream()), "nirc_probe_mfma")
    per_mfma = 2048 if precision == NIRC_FP32 else 16384
    return 8 * iters * 4 * blocks * per_mfma


def nirc_probe_atomics(lanes_per_line: int, reps: int, blocks: int, buf: torch.Tensor):
    """Atomics microbenchmark on the current stream (buf: int64 device tensor, length a power of
    two); returns the number of adds (the caller times the launch)."""
    _check(lib().nirc_probe_atomics(lanes_per_line, reps, blocks, _ptr(buf), buf.numel(), _stream()),
           "nirc_probe_atomics")
    return blocks * 256 * reps


NIRC_STATIC_MAX_BATCH = 2048


def nirc_train_step_static(model: Model, points: Points, queries: Queries, target: torch.Tensor, loss=None):
    """nirc_train_step on the library's static scratch (no workspace needed, nothing allocated;
    batches up to NIRC_STATIC_MAX_BATCH; calls on one GPU must not overlap)."""
    _check(lib().nirc_train_step_static(model.handle, points.c(), queries.c(), _ptr(target), _ptr(loss), _stream()),
           "nirc_train_step_static")
    return loss


TLMC_CHEB_COEFFS = 128
TLMC_STATS = 8


def tlmc_reference_occluded(points: Points, lobes, n_nodes: int = 64) -> torch.Tensor:
    """Quadrature reference of the occluded scene's integral, [P, 3] FP64."""
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    F = torch.empty((points.count, 3), dtype=torch.float64, device=points.t[0].device)
    _check(lib().tlmc_reference_occluded(points.c(), ctypes.byref(L), n_nodes, _ptr(F), _stream()),
           "tlmc_reference_occluded")
    return F


def tlmc_reference_table(lobes, device="cuda") -> torch.Tensor:
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    t = torch.empty((4, TLMC_CHEB_COEFFS), dtype=torch.float64, device=device)
    _check(lib().tlmc_reference_table(ctypes.byref(L), _ptr(t), _stream()), "tlmc_reference_table")
    return t


def tlmc_reference(points: Points, lobes, table: torch.Tensor) -> torch.Tensor:
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    F = torch.empty((points.count, 3), dtype=torch.float64, device=table.device)
    _check(lib().tlmc_reference(points.c(), ctypes.byref(L), _ptr(table), _ptr(F), _stream()), "tlmc_reference")
    return F


class FrameStats:
    """Reusable scratch + output for tlmc_frame_stats."""

    def __init__(self, device="cuda"):
        nb = int(lib().tlmc_frame_stats_scratch_bytes())
        self.scratch = torch.empty(nb // 8, dtype=torch.float64, device=device)
        self.stats = torch.zeros(TLMC_STATS, dtype=torch.float64, device=device)


def tlmc_frame_stats(points: Points, lobes, table: torch.Tensor, est_tl, est_c=None, est_r=None,
                     eps: float = 1e-2, fs: FrameStats | None = None) -> torch.Tensor:
    """FP64 stats [8]: sums of relative squared errors, count, and MRSE (index 4)."""
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    fs = fs or FrameStats(table.device)
    _check(lib().tlmc_frame_stats(points.c(), ctypes.byref(L), _ptr(table), _ptr(est_tl), _ptr(est_c), _ptr(est_r),
                                  eps, _ptr(fs.scratch), _ptr(fs.stats), _stream()), "tlmc_frame_stats")
    return fs.stats


def tlmc_accumulate(values: torch.Tensor, s: torch.Tensor, s2: torch.Tensor):
    _check(lib().tlmc_accumulate(_ptr(values), values.numel(), _ptr(s), _ptr(s2), _stream()), "tlmc_accumulate")


def nirc_train_frame(model: Model, points: Points, lobes, batch: int, steps: int, seed: int, frame: int,
                     loss: torch.Tensor | None = None):
    """steps x (training samples + train step) in one native call; samples live in the workspace."""
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    _check(lib().nirc_train_frame(model.handle, points.c(), ctypes.byref(L), batch, steps, seed, frame, _ptr(loss),
                                  _stream()), "nirc_train_frame")


TLMC_BATCH_MAX_REQUESTS = 64


class Batch:
    """A reusable device work list for tlmc_estimate_batch (continuous batching of several
    streams' frames into one persistent launch)."""

    def __init__(self, device="cuda"):
        self.nbytes = int(lib().tlmc_batch_bytes())
        self.host = torch.zeros(self.nbytes, dtype=torch.uint8).pin_memory()
        self.dev = torch.zeros(self.nbytes, dtype=torch.uint8, device=device)
        self.width = None
        self.precision = None
        self.output = None
        self._keep = []
        self._copied = None

    def set(self, requests):
        """requests: list of dicts with model, points, lobes, n_cache, seed, frame, out_tl[, out_c, out_r,
        residual].
        Writes the work list to the device buffer on the current stream."""
        n = len(requests)
        if self._copied is not None:
            self._copied.synchronize()   # the previous list's host-to-device copy has run
        arr = (_Request * n)()
        self._keep = []
        for i, r in enumerate(requests):
            lb = r.get("lobes")
            L = lb if isinstance(lb, Lobes) else (Lobes() if lb is None else lobes_struct(lb))
            rr = r.get("residual")
            if lb is None and rr is None:
                raise NircError("a request needs lobes or residual radiance")
            arr[i] = _Request(r["model"].handle.value, r["points"].c(), L, r["n_cache"], r["seed"], r["frame"],
                              None if rr is None else rr.data_ptr(),
                              r["out_tl"].data_ptr(), _ptr(r.get("out_c")) and r["out_c"].data_ptr(),
                              _ptr(r.get("out_r")) and r["out_r"].data_ptr())
            self._keep.append(r)
        _check(lib().tlmc_batch_build(arr, n, ctypes.c_void_p(self.host.data_ptr())), "tlmc_batch_build")
        self.width = requests[0]["model"].width
        self.precision = requests[0]["model"].cfg.precision
        self.output = requests[0]["model"].cfg.output
        self.dev.copy_(self.host, non_blocking=True)
        self._copied = torch.cuda.Event()
        self._copied.record()

    def launch(self):
        _check(lib().tlmc_estimate_batch(ctypes.c_void_p(self.dev.data_ptr()), self.width, self.precision, self.output,
                                         _stream()),
               "tlmc_estimate_batch")


NIRC_TRAIN_BATCH_MAX_REQUESTS = 64


class TrainBatch:
    """A reusable device work list for nirc_train_frame_batch (one frame's training of several
    streams' caches in one set of launches)."""

    def __init__(self, max_batch: int, device="cuda"):
        self.nbytes = int(lib().nirc_train_list_bytes())
        self.host = torch.zeros(self.nbytes, dtype=torch.uint8).pin_memory()
        self.dev = torch.zeros(self.nbytes, dtype=torch.uint8, device=device)
        self.max_batch = int(max_batch)
        self.precision = None
        self._keep = []
        self._copied = None

    def set(self, requests):
        """requests: list of dicts with model, points, lobes, batch, seed, frame.  Writes the work
        list to the device buffer on the current stream."""
        n = len(requests)
        if self._copied is not None:
            self._copied.synchronize()   # the previous list's host-to-device copy has run
        arr = (_TrainRequest * n)()
        self._keep = list(requests)
        for i, r in enumerate(requests):
            lb = r["lobes"]
            L = lb if isinstance(lb, Lobes) else lobes_struct(lb)
            arr[i] = _TrainRequest(r["model"].handle.value, r["points"].c(), L, int(r["batch"]), int(r["seed"]),
                                   int(r["frame"]))
        _check(lib().nirc_train_list_build(arr, n, self.max_batch, ctypes.c_void_p(self.host.data_ptr())),
               "nirc_train_list_build")
        self.precision = requests[0]["model"].cfg.precision
        self.dev.copy_(self.host, non_blocking=True)
        self._copied = torch.cuda.Event()
        self._copied.record()

    def launch(self, steps: int, precision: int | None = None):
        prec = self.precision if precision is None else precision
        _check(lib().nirc_train_frame_batch(ctypes.c_void_p(self.dev.data_ptr()), steps, prec, self.max_batch,
                                            _stream()), "nirc_train_frame_batch")


class NircFunction(torch.autograd.Function):
    """y = cache(w; points, queries) with the hand-written backward (weight gradients only).

    forward loads w into `model` with nirc_set_weights (which also resets that model's Adam
    state, so use a model dedicated to evaluation) and runs nirc_infer; backward runs
    nirc_backward with the upstream gradient.
    """

    @staticmethod
    def forward(ctx, w, model, points, queries):
        _check(lib().nirc_set_weights(model.handle, _ptr(w.contiguous()), _stream()), "nirc_set_weights")
        ctx.model, ctx.points, ctx.queries = model, points, queries
        return nirc_infer(model, points, queries)

    @staticmethod
    def backward(ctx, dy):
        g = nirc_backward(ctx.model, ctx.points, ctx.queries, dy.contiguous())
        return g, None, None, None


# ------------------------------------------------------------------------------------------
# The hash-grid cache input (hash grid on x, spherical harmonics of w, identity / one-blob phi)

def make_hash_grid(log2_table: int = 18, base_res: int = 16, growth: float = 1.5) -> HashGrid:
    return HashGrid(log2_table, base_res, growth)


def nirc_hash_entries(grid: HashGrid) -> int:
    return int(lib().nirc_hash_entries(ctypes.byref(grid)))


def nirc_hash_n_params(grid: HashGrid) -> int:
    return int(lib().nirc_hash_n_params(ctypes.byref(grid)))


def nirc_hash_levels(grid: HashGrid):
    """(resolution [12], first entry [12], dense flag [12]) as numpy arrays."""
    res = np.zeros(12, np.int32)
    off = np.zeros(12, np.int64)
    dense = np.zeros(12, np.int32)
    _check(lib().nirc_hash_levels(ctypes.byref(grid), res.ctypes.data, off.ctypes.data, dense.ctypes.data),
           "nirc_hash_levels")
    return res, off, dense


class HashModel:
    """A hash-grid cache model (width 64, 16-bit layer products) over torch-allocated memory."""

    def __init__(self, init_w, cfg: Config | None = None, grid: HashGrid | None = None, max_batch: int = 65536,
                 device="cuda"):
        self.cfg = cfg or make_config(precision=NIRC_BF16)
        self.grid = grid or make_hash_grid()
        self.n_params = nirc_hash_n_params(self.grid)
        sb = int(lib().nirc_hash_state_bytes(ctypes.byref(self.cfg), ctypes.byref(self.grid)))
        if sb == 0 or self.n_params == 0:
            raise NircError("unsupported hash-grid configuration")
        self.state = torch.empty(sb, dtype=torch.uint8, device=device)
        wb = int(lib().nirc_hash_workspace_bytes(ctypes.byref(self.cfg), ctypes.byref(self.grid), max_batch)) \
            if max_batch > 0 else 0
        self.workspace = torch.empty(wb, dtype=torch.uint8, device=device) if wb else None
        w = init_w if isinstance(init_w, torch.Tensor) else _dev_f32(init_w, device)
        assert w.numel() == self.n_params
        self._w0 = w.contiguous()
        h = _vp()
        _check(lib().nirc_hash_create(ctypes.byref(self.cfg), ctypes.byref(self.grid), _ptr(self.state), sb,
                                      _ptr(self.workspace), wb, _ptr(self._w0), _stream(), ctypes.byref(h)),
               "nirc_hash_create")
        self.handle = h

    def __del__(self):
        h = getattr(self, "handle", None)
        if h is not None and _lib is not None:
            _lib.nirc_hash_destroy(h)
            self.handle = None

    def set_weights(self, w: torch.Tensor):
        self._w0 = w.contiguous()
        _check(lib().nirc_hash_set_weights(self.handle, _ptr(self._w0), _stream()), "nirc_hash_set_weights")

    def get_weights(self) -> torch.Tensor:
        out = torch.empty(self.n_params, dtype=torch.float32, device=self.state.device)
        _check(lib().nirc_hash_get_weights(self.handle, _ptr(out), _stream()), "nirc_hash_get_weights")
        return out

    def get_state(self) -> torch.Tensor:
        """The whole training state as a device byte tensor (checkpoint)."""
        out = torch.empty(self.state.numel(), dtype=torch.uint8, device=self.state.device)
        _check(lib().nirc_hash_get_state(self.handle, _ptr(out), out.numel(), _stream()), "nirc_hash_get_state")
        return out

    def set_state(self, blob: torch.Tensor):
        """Restore a state written by get_state of a model with the same grid (resume)."""
        b = blob.to(self.state.device).contiguous()
        _check(lib().nirc_hash_set_state(self.handle, _ptr(b), b.numel(), _stream()), "nirc_hash_set_state")
        torch.cuda.current_stream().synchronize()   # b may be a temporary

    def read_flags(self) -> int:
        return int(lib().nirc_hash_read_flags(self.handle, _stream()))


def nirc_hash_infer(model: HashModel, points: Points, queries: Queries) -> torch.Tensor:
    out = torch.empty((queries.count, 3), dtype=torch.float32, device=points.t[0].device)
    _check(lib().nirc_hash_infer(model.handle, points.c(), queries.c(), _ptr(out), _stream()), "nirc_hash_infer")
    return out


def nirc_hash_estimate(model: HashModel, points: Points, lobes, n_cache: int, seed: int, frame: int,
                       parts: bool = False, out=None, residual=None):
    """Two-level estimate per point with the hash-grid cache; F_tl, or (F_tl, F_c, F_r)."""
    dev = points.t[0].device
    L = None if lobes is None else (lobes if isinstance(lobes, Lobes) else lobes_struct(lobes))
    tl = out if out is not None else torch.empty((points.count, 3), dtype=torch.float32, device=dev)
    c = torch.empty_like(tl) if parts else None
    r = torch.empty_like(tl) if parts else None
    if residual is not None:
        assert residual.dtype == torch.float32 and residual.is_contiguous() and residual.numel() == 3 * points.count
    _check(lib().nirc_hash_estimate(model.handle, points.c(), None if L is None else ctypes.byref(L), n_cache, seed,
                                    frame, _ptr(residual), _ptr(tl), _ptr(c), _ptr(r), _stream()),
           "nirc_hash_estimate")
    return (tl, c, r) if parts else tl


def nirc_hash_loss_grad(model: HashModel, points: Points, queries: Queries, target: torch.Tensor):
    """(loss [1], gradient [n_params]) of a batch, without an update."""
    grad = torch.empty(model.n_params, dtype=torch.float32, device=points.t[0].device)
    loss = torch.empty(1, dtype=torch.float32, device=points.t[0].device)
    t = target.contiguous()
    _check(lib().nirc_hash_loss_grad(model.handle, points.c(), queries.c(), _ptr(t), _ptr(grad), _ptr(loss),
                                     _stream()), "nirc_hash_loss_grad")
    return loss, grad


def nirc_hash_adam_step(model: HashModel, grad: torch.Tensor):
    _check(lib().nirc_hash_adam_step(model.handle, _ptr(grad.contiguous()), _stream()), "nirc_hash_adam_step")


def nirc_hash_train_step(model: HashModel, points: Points, queries: Queries, target: torch.Tensor, loss=None):
    t = target.contiguous()
    _check(lib().nirc_hash_train_step(model.handle, points.c(), queries.c(), _ptr(t), _ptr(loss), _stream()),
           "nirc_hash_train_step")


def nirc_hash_train_frame(model: HashModel, points: Points, lobes, batch: int, steps: int, seed: int, frame: int,
                          loss=None):
    """One frame of online training of a hash-grid model (steps x generated batch + train step)."""
    L = lobes if isinstance(lobes, Lobes) else lobes_struct(lobes)
    _check(lib().nirc_hash_train_frame(model.handle, points.c(), ctypes.byref(L), batch, steps, seed, frame,
                                       _ptr(loss), _stream()), "nirc_hash_train_frame")
