#!/usr/bin/env python3
"""Benchmark of one frame of the NIRC two-level Monte Carlo hot path on one MI355X.

A step is one frame of the dynamic 1080p scene (lobe axes rotate one degree per frame):
  tlmc_estimate (N = 16 cache directions + 1 residual per point)      gather .. combine
  tlmc_frame_stats (FP64 MRSE against the exact integral)             frame statistics
  4 x (tlmc_train_batch + nirc_train_step), batch 65,536               training + Adam
All inputs are resident in HBM before timing starts.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import collections
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "NIRC queries/s + ms/frame at 1080p N=16; BF16 vs FP32 at equal MRSE"
PEAK_FP32_MFMA = 157.3e12      # MI355X dense FP32 matrix peak, FLOP/s
PEAK_BF16_MFMA = 2.5e15        # MI355X dense BF16/FP16 matrix peak, FLOP/s
PEAK_HBM = 8.0e12              # bytes/s
# HBM bytes per launch of k_tlmc_f32 in the frame configuration (1080p, N = 16, F_tl + F_c + F_r
# written), from FETCH_SIZE x 2.0 + WRITE_SIZE (factors from a plain 512 MiB copy); recorded in
# profiles/k_tlmc_hbm_counters_1080p_n16.md and to be measured again whenever the kernel changes.
TRAFFIC_K_TLMC_F32 = 134192896


def algorithmic_flops_estimate(P: int, N: int, W: int) -> float:
    """Per launch of the fused estimator: surface projection once per point plus, per query,
    the direction columns of layer 1, three hidden layers and the output layer."""
    surface = 2 * 112 * W
    per_query = 2 * (48 * W + 3 * W * W + 3 * W)
    return float(P) * (surface + (N + 1) * per_query)


def algorithmic_flops_train(B: int, W: int) -> float:
    """One training step: forward (160-wide input), weight gradients and deltas (no input grads)."""
    fwd = 2 * (160 * W + 3 * W * W + 3 * W)
    dw = fwd
    delta = 2 * (3 * W * W + 3 * W)
    return float(B) * (fwd + dw + delta)


def cpu_baseline(pts, lobes_for, w0, W, N, B, steps_per_frame, target_s=12.0, target_1core_s=6.0):
    """The FP64 oracle on a bounded sample of the same frame: a seeded subset of points and a
    proportional share of the training batch; reported as queries/s of the whole frame, on all
    the oracle's threads and on one."""
    import numpy as np
    import oracle

    P = pts.count
    rng = np.random.default_rng(1234)

    def run(n_pts):
        sel = np.sort(rng.choice(P, n_pts, replace=False))
        sub = pts.subset(sel)
        b = max(1, int(round(B * n_pts / P)))
        lob = lobes_for(0)
        t0 = time.perf_counter()
        oracle.estimate(sub, lob, w0, W, N, 2, 0)
        w = w0.astype(np.float64).copy()
        m = np.zeros_like(w)
        v = np.zeros_like(w)
        for s in range(steps_per_frame):
            idx, d, t = oracle.train_batch(sub, lob, b, 2, 0, s)
            _, g = oracle.loss_grad(sub, idx, d, t, w, W)
            oracle.adam(w, m, v, g, s + 1)
        return time.perf_counter() - t0, b

    threads = oracle.threads()

    def cfg1_frame():
        # the small configuration's whole frame: 64 x 64 points, N = 8, one Adam step on 4096
        # samples, width 64
        from paper_2412_04634_amd import workload as wl
        p1 = wl.make_points(1, 4096)
        l1 = wl.make_lobes(1).packed()
        w1 = wl.make_weights(1, 64).astype(np.float64)
        t0 = time.perf_counter()
        oracle.estimate(p1, l1, w1, 64, 8, 1, 0)
        idx, d, t = oracle.train_batch(p1, l1, 4096, 1, 0, 0)
        _, g = oracle.loss_grad(p1, idx, d, t, w1, 64)
        oracle.adam(w1, np.zeros_like(w1), np.zeros_like(w1), g, 1)
        return (time.perf_counter() - t0) * 1e3

    cfg1_ms = cfg1_frame()
    t_small, _ = run(512)
    n = int(min(P, max(512, 512 * target_s / max(t_small, 1e-3))))
    t, b = run(n)
    oracle.set_threads(1)
    try:
        cfg1_ms_1 = cfg1_frame()
        t1_small, _ = run(64)
        n1 = int(min(P, max(64, 64 * target_1core_s / max(t1_small, 1e-3))))
        t1, b1 = run(n1)
    finally:
        oracle.set_threads(threads)
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": n * (N + 1) / t, "unit": "queries/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "small_frame_ms": {"all_threads": cfg1_ms, "one_core": cfg1_ms_1,
                               "frame": "4096 points, N = 8 + 1 residual, 1 Adam step of 4096 samples, width 64"},
            "sample": f"{n} of {P} points (seeded subset) x {N}+1 queries + {steps_per_frame} training "
                      f"steps of {b} samples (batch scaled by the same fraction); {t:.1f} s",
            "one_core": {"value": n1 * (N + 1) / t1, "unit": "queries/s", "cores": 1,
                         "sample": f"{n1} points, training batch {b1}; {t1:.1f} s"}}


def mfma_probe(nirc):
    """The matrix rate a kernel of independent MFMA chains reaches here (1024 workgroups, 4 waves
    per SIMD; second launch of each), per precision, and the same BF16 kernel with 32 or 64 FP32
    FMAs per 8 MFMAs in each wave: the measured peak the roofline fractions are also quoted
    against, and whether VALU work hides under the MFMAs."""
    import torch
    sink = torch.empty(1024 * 256, dtype=torch.float32, device="cuda")
    out = {}

    def timed(prec, iters, fmas):
        t = None
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            flops = nirc.nirc_probe_mfma(prec, iters, fmas, sink)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3
        return flops, t

    for name, prec, iters in (("fp32", 0, 2048), ("bf16", 1, 4096), ("fp16", 2, 4096)):
        flops, t = timed(prec, iters, 0)
        out[name] = {"tflops": flops / t / 1e12, "ms": t * 1e3,
                     "frac_of_vendor_peak": flops / t / (PEAK_FP32_MFMA if prec == 0 else PEAK_BF16_MFMA)}
    _, t0 = timed(1, 4096, 0)
    for fm in (32, 64):
        _, t = timed(1, 4096, fm)
        out[f"bf16_plus_{fm}_fma_per_8_mfma"] = {"ms": t * 1e3, "ratio_to_mfma_only": t / t0}
    # 64-bit integer atomic adds (the hash-grid gradient scatter) into a 32 MB buffer, by lanes
    # per 128-byte line: 4096 workgroups x 256 threads x 16 adds
    buf = torch.zeros(1 << 22, dtype=torch.int64, device="cuda")
    for lpl in (1, 4, 16):
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            adds = nirc.nirc_probe_atomics(lpl, 16, 4096, buf)
            e1.record()
            torch.cuda.synchronize()
            t = e0.elapsed_time(e1) * 1e-3
        out[f"atomic_add_u64_{lpl}_lanes_per_line"] = {"g_adds_per_s": adds / t / 1e9, "ms": t * 1e3}
    return out


def precision_compare(nirc, model32, dp, lobes_for, table, fs, P, N, W, seed, frame, reps, B, S):
    """BF16 and FP16 estimates with the FP32 model's current weights, same seed and frame:
    time per launch (HIP events on the launch stream) and MRSE against the exact integral; and
    one frame of training (S steps of B samples) at each precision, on a copy of the model."""
    import torch
    stream = torch.cuda.current_stream()
    w = model32.get_weights()
    lob = nirc.lobes_struct(lobes_for(frame))
    out = {}
    for name, prec in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
        m = model32 if prec == 0 else nirc.Model(w, cfg=nirc.make_config(precision=prec), max_batch=0)
        tl = torch.empty((P, 3), dtype=torch.float32, device="cuda")
        nirc.tlmc_estimate(m, dp, lob, N, seed, frame, out=tl)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            nirc.tlmc_estimate(m, dp, lob, N, seed, frame, out=tl)
        ev[1].record(stream)
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        mrse = float(nirc.tlmc_frame_stats(dp, lob, table, tl, fs=fs)[4].item())
        flops = algorithmic_flops_estimate(P, N, W)
        peak = PEAK_FP32_MFMA if prec == 0 else PEAK_BF16_MFMA
        mt = nirc.Model(w, cfg=nirc.make_config(precision=prec), max_batch=B)
        nirc.nirc_train_frame(mt, dp, lob, B, S, seed, frame)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for r in range(reps):
            nirc.nirc_train_frame(mt, dp, lob, B, S, seed, frame + 1 + r)
        ev[1].record(stream)
        torch.cuda.synchronize()
        tt = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
        out[name] = {"ms_estimate": t * 1e3, "queries_per_s": P * (N + 1) / t, "mrse": mrse,
                     "roofline": {"bound": "mfma", "achieved": flops / t / 1e12, "peak": peak / 1e12,
                                  "unit": "TFLOP/s", "frac": flops / t / peak},
                     "ms_train_frame": tt * 1e3, "train_samples_per_s": S * B / tt,
                     "train_tflops": algorithmic_flops_train(B, W) * S / tt / 1e12}
    for name in ("bf16", "fp16"):
        out[name]["speedup_vs_fp32"] = out["fp32"]["ms_estimate"] / out[name]["ms_estimate"]
        out[name]["mrse_rel_diff_vs_fp32"] = (out[name]["mrse"] - out["fp32"]["mrse"]) / out["fp32"]["mrse"]
    return out


def precision_form(nirc, w64, dp, lob_packed, table, fs, P, seed, frame, reps=3):
    """The precision matrix: N in {4, 16, 64} x width {64, 128} x {FP32, BF16, FP16} estimates
    of one 1080p frame on identical weights (width 64: the benchmark's trained FP32 cache;
    width 128: an FP32 cache trained for 20 frames here).  Per entry: time per launch,
    queries/s, MFMA fraction, MRSE against the exact integral, and rel-L2 of F_tl against the
    FP32 result on the same weights and directions."""
    import torch
    from paper_2412_04634_amd import workload as wl
    stream = torch.cuda.current_stream()
    lob = nirc.lobes_struct(lob_packed)
    rows = []
    for W in (64, 128):
        if W == 64:
            w = w64
        else:
            m128 = nirc.Model(wl.make_weights(seed, W), cfg=nirc.make_config(width=W), max_batch=65536)
            for f in range(20):
                nirc.nirc_train_frame(m128, dp, lob, 65536, 4, seed, f)
            w = m128.get_weights()
            del m128
        for N in (4, 16, 64):
            ref = None
            for name, prec in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
                m = nirc.Model(w, cfg=nirc.make_config(width=W, precision=prec), max_batch=0)
                tl = torch.empty((P, 3), dtype=torch.float32, device="cuda")
                nirc.tlmc_estimate(m, dp, lob, N, seed, frame, out=tl)
                ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
                torch.cuda.synchronize()
                ev[0].record(stream)
                for _ in range(reps):
                    nirc.tlmc_estimate(m, dp, lob, N, seed, frame, out=tl)
                ev[1].record(stream)
                torch.cuda.synchronize()
                t = ev[0].elapsed_time(ev[1]) * 1e-3 / reps
                mrse = float(nirc.tlmc_frame_stats(dp, lob, table, tl, fs=fs)[4].item())
                if ref is None:
                    ref = tl.clone()
                flops = algorithmic_flops_estimate(P, N, W)
                peak = PEAK_FP32_MFMA if prec == 0 else PEAK_BF16_MFMA
                rows.append({"width": W, "n_cache": N, "precision": name, "ms_estimate": t * 1e3,
                             "queries_per_s": P * (N + 1) / t, "mfma_frac": flops / t / peak, "mrse": mrse,
                             "rel_l2_vs_fp32": float((tl - ref).norm() / ref.norm())})
                del m
    return rows


def precision_trained(nirc, w0, dp, lobes_for, table, fs, P, N, seed, frames, B, S):
    """Each precision trains its own cache from the same initial weights over the same rotating
    frames (estimate with W(f), then S Adam steps of B samples): MRSE of the last frame's estimate
    against the exact integral, and the average estimate / training time per frame."""
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    for name, prec in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
        m = nirc.Model(w0, cfg=nirc.make_config(precision=prec), max_batch=B)
        tl = torch.empty((P, 3), dtype=torch.float32, device="cuda")
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(frames)]
        mrse = None
        for f in range(frames):
            lob = nirc.lobes_struct(lobes_for(f))
            ev[f][0].record(stream)
            nirc.tlmc_estimate(m, dp, lob, N, seed, f, out=tl)
            ev[f][1].record(stream)
            if f == frames - 1:
                mrse = float(nirc.tlmc_frame_stats(dp, lob, table, tl, fs=fs)[4].item())
            nirc.nirc_train_frame(m, dp, lob, B, S, seed, f)
            ev[f][2].record(stream)
        torch.cuda.synchronize()
        t_est = sum(e[0].elapsed_time(e[1]) for e in ev[1:]) / (frames - 1)
        t_all = sum(e[0].elapsed_time(e[2]) for e in ev[1:]) / (frames - 1)
        out[name] = {"mrse_last_frame": mrse, "ms_estimate": t_est, "ms_estimate_plus_train": t_all}
        del m
    for name in ("bf16", "fp16"):
        out[name]["mrse_rel_diff_vs_fp32"] = (out[name]["mrse_last_frame"] - out["fp32"]["mrse_last_frame"]) / \
            out["fp32"]["mrse_last_frame"]
    out["frames"] = frames
    return out


def train_convergence(nirc, dp, lobes_for, W, seed, frames=300, batches=(1 << 16, 1 << 18, 1 << 20),
                      precision=0):
    """The differentiation workload: online training only, 4 Adam steps per frame on the rotating
    1080p field for each batch size; every 30 frames the cache's relative L2 error against the
    field on a fixed-size probe of fresh samples of that frame (65,536 queries), and the training
    throughput."""
    import torch
    from paper_2412_04634_amd import workload as wl
    stream = torch.cuda.current_stream()
    out = {}
    for B in batches:
        m = nirc.Model(wl.make_weights(seed, W), cfg=nirc.make_config(width=W, precision=precision), max_batch=B)
        curve = []
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t_train = 0.0
        for f in range(frames):
            lob = nirc.lobes_struct(lobes_for(f))
            if f % 30 == 0 or f == frames - 1:
                q, tgt = nirc.tlmc_train_batch(dp, lob, 65536, seed + 7919, f, 0)
                y = nirc.nirc_infer(m, dp, q)
                curve.append([f, float((y - tgt).norm() / tgt.norm())])
            ev[0].record(stream)
            nirc.nirc_train_frame(m, dp, lob, B, 4, seed, f)
            ev[1].record(stream)
            ev[1].synchronize()
            t_train += ev[0].elapsed_time(ev[1]) * 1e-3
        out[str(B)] = {"cache_rel_l2": curve, "ms_train_frame": t_train / frames * 1e3,
                       "train_samples_per_s": 4 * B * frames / t_train,
                       "train_tflops": algorithmic_flops_train(B, W) * 4 * frames / t_train / 1e12}
        del m
    return out


def biased_compare(nirc, model32, dp, lobes_for, table, fs, P, N, seed, frame, reps):
    """The biased estimator with the balanced termination heuristic beside the unbiased two-level
    estimator, on the FP32 model's current weights at FP32 and BF16: time per call (fused
    estimator + decision kernel), fraction of continued paths, MRSE of both against the exact
    integral."""
    import torch
    stream = torch.cuda.current_stream()
    w = model32.get_weights()
    lob = nirc.lobes_struct(lobes_for(frame))
    out = {}
    for name, prec in (("fp32", 0), ("bf16", 1)):
        m = model32 if prec == 0 else nirc.Model(w, cfg=nirc.make_config(precision=prec), max_batch=0)
        b, c, cont = nirc.tlmc_estimate_biased(m, dp, lob, N, seed, frame)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            nirc.tlmc_estimate_biased(m, dp, lob, N, seed, frame, out=b)
        ev[1].record(stream)
        torch.cuda.synchronize()
        tl = nirc.tlmc_estimate(m, dp, lob, N, seed, frame)
        mrse_b = float(nirc.tlmc_frame_stats(dp, lob, table, b, fs=fs)[4].item())
        mrse_u = float(nirc.tlmc_frame_stats(dp, lob, table, tl, fs=fs)[4].item())
        out[name] = {"ms_biased": ev[0].elapsed_time(ev[1]) / reps, "continued_fraction": float(cont.float().mean()),
                     "mrse_biased": mrse_b, "mrse_unbiased": mrse_u}
    return out


def visibility_compare(nirc, w0, dp, lobes_for, P, N, seed, frames, B, S):
    """The occluded (environment-lit) scene: a visibility cache (sigmoid outputs times the known
    radiance) against a radiance cache learning V L, each trained from the same weights over the
    same rotating frames.  On the last frame: MRSE of the two-level estimate and of the cache
    level alone against the 64-node quadrature of V L, the residual's relative second moment, and
    the GPU time per estimate and per training frame.  (The MRSE of this comparison is computed
    with torch in FP64 from the estimate and the reference, as the frame statistics' closed form
    covers the unoccluded scene only.)"""
    import torch
    stream = torch.cuda.current_stream()
    lob = nirc.lobes_struct(lobes_for(frames))
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record(stream)
    F = nirc.tlmc_reference_occluded(dp, lob, 64)
    ev[1].record(stream)
    torch.cuda.synchronize()
    out = {"ms_reference_quadrature": ev[0].elapsed_time(ev[1])}
    den = F * F + 1e-2
    for name, mode in (("visibility_cache", 1), ("radiance_cache", 2)):
        m = nirc.Model(w0, cfg=nirc.make_config(output=mode), max_batch=B)
        t_train = 0.0
        for f in range(frames):
            ev[0].record(stream)
            nirc.nirc_train_frame(m, dp, nirc.lobes_struct(lobes_for(f)), B, S, seed, f)
            ev[1].record(stream)
            ev[1].synchronize()
            t_train += ev[0].elapsed_time(ev[1])
        tl, c, r = nirc.tlmc_estimate(m, dp, lob, N, seed, frames, parts=True)
        ev[0].record(stream)
        nirc.tlmc_estimate(m, dp, lob, N, seed, frames, out=tl)
        ev[1].record(stream)
        torch.cuda.synchronize()
        out[name] = {"mrse": float(((tl.double() - F) ** 2 / den).mean()),
                     "mrse_cache_only": float(((c.double() - F) ** 2 / den).mean()),
                     "residual_rel_second_moment": float((r.double() ** 2 / den).mean()),
                     "ms_estimate": ev[0].elapsed_time(ev[1]), "ms_train_frame": t_train / frames}
        del m
    out["frames"] = frames
    return out


def loss_variants(nirc, w0, dp, lobes_for, table, fs, P, N, seed, frames, B, S):
    """The three training losses of the optimisation section (relative L2, plain L2, residual
    variance), each training its own FP32 cache from the same weights over the same rotating
    frames: MRSE of the two-level estimate and of the cache level alone on the last frame, the
    cache's relative L2 error on a probe of fresh samples, and the training time per frame."""
    import torch
    stream = torch.cuda.current_stream()
    out = {}
    for name, kind in (("rel_l2", 0), ("l2", 1), ("variance", 2)):
        m = nirc.Model(w0, cfg=nirc.make_config(loss=kind), max_batch=B)
        tl = torch.empty((P, 3), dtype=torch.float32, device="cuda")
        c = torch.empty_like(tl)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        t_train = 0.0
        for f in range(frames):
            lob = nirc.lobes_struct(lobes_for(f))
            ev[0].record(stream)
            nirc.nirc_train_frame(m, dp, lob, B, S, seed, f)
            ev[1].record(stream)
            ev[1].synchronize()
            t_train += ev[0].elapsed_time(ev[1])
        lob = nirc.lobes_struct(lobes_for(frames))
        nirc._check(nirc.lib().tlmc_estimate(m.handle, dp.c(), nirc.ctypes.byref(lob), N, seed, frames, None,
                                             nirc._ptr(tl), nirc._ptr(c), None, nirc._stream()), "tlmc_estimate")
        st = nirc.tlmc_frame_stats(dp, lob, table, tl, c, fs=fs)
        q, tgt = nirc.tlmc_train_batch(dp, lob, 65536, seed + 7919, frames, 0)
        y = nirc.nirc_infer(m, dp, q)
        out[name] = {"mrse": float(st[4].item()), "mrse_cache_only": float(st[5].item()),
                     "cache_rel_l2": float((y - tgt).norm() / tgt.norm()), "ms_train_frame": t_train / frames,
                     "flags": m.read_flags()}
        del m
    out["frames"] = frames
    return out


def algorithmic_flops_hash(P: int, N: int, W: int = 64) -> float:
    """Hash-grid model: 39 surface inputs (24 grid values + 15 surface values) projected once per
    point, then per query the 25 SH inputs, three hidden layers and the output layer."""
    return float(P) * (2 * 39 * W + (N + 1) * 2 * (25 * W + 3 * W * W + 3 * W))


def hash_grid_compare(nirc, w0, dp, lobes_for, table, fs, P, N, seed, frames, B, S, reps=20, pts_host=None):
    """The paper's own cache input (hash grid on x, spherical harmonics of w, one-blob surface
    values) against the frequency input, both BF16, and the hash-grid cache trained and evaluated
    in FP32, each trained online from its initial weights over the same rotating frames: time per estimate (N + 1 queries per point) and per training
    frame, and on the last frame the MRSE of the two-level estimate and of the cache level alone
    against the closed form, and the cache's relative L2 error on fresh samples (also before
    frames 0, 5, 10, 25 and 50, as a convergence curve)."""
    import torch
    from paper_2412_04634_amd import workload as wl
    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    grid = nirc.make_hash_grid()
    wh = wl.make_hash_weights(seed, 64, 2 * nirc.nirc_hash_entries(grid))
    models = {"frequency_bf16": nirc.Model(w0, cfg=nirc.make_config(precision=1), max_batch=B),
              "hash_grid_bf16": nirc.HashModel(wh, cfg=nirc.make_config(precision=1), grid=grid, max_batch=B),
              "hash_grid_fp32": nirc.HashModel(wh, cfg=nirc.make_config(precision=0), grid=grid, max_batch=B)}
    out = {"grid": {"levels": 12, "features": 2, "log2_table": grid.log2_table, "base_res": grid.base_res,
                    "growth": grid.growth, "entries": nirc.nirc_hash_entries(grid),
                    "table_mb": 8 * nirc.nirc_hash_entries(grid) / 1e6}}
    tl = torch.empty((P, 3), dtype=torch.float32, device="cuda")
    c = torch.empty_like(tl)
    checkpoints = [0, 5, 10, 25, 50, frames]
    for name, m in models.items():
        is_hash = isinstance(m, nirc.HashModel)
        t_train = 0.0
        curve = []

        def probe(f):
            lob_p = nirc.lobes_struct(lobes_for(f))
            qp, tp = nirc.tlmc_train_batch(dp, lob_p, 65536, seed + 7919, f, 0)
            yp = nirc.nirc_hash_infer(m, dp, qp) if is_hash else nirc.nirc_infer(m, dp, qp)
            curve.append([f, float((yp - tp).norm() / tp.norm())])

        for f in range(frames):
            if f in checkpoints:
                probe(f)
            lob = nirc.lobes_struct(lobes_for(f))
            ev[0].record(stream)
            if is_hash:
                nirc.nirc_hash_train_frame(m, dp, lob, B, S, seed, f)
            else:
                nirc.nirc_train_frame(m, dp, lob, B, S, seed, f)
            ev[1].record(stream)
            ev[1].synchronize()
            t_train += ev[0].elapsed_time(ev[1])
        lob = nirc.lobes_struct(lobes_for(frames))
        est = (lambda: nirc.nirc_hash_estimate(m, dp, lob, N, seed, frames, out=tl)) if is_hash else \
            (lambda: nirc.tlmc_estimate(m, dp, lob, N, seed, frames, out=tl))
        for _ in range(3):
            est()
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            est()
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        if is_hash:
            nirc._check(nirc.lib().nirc_hash_estimate(m.handle, dp.c(), nirc.ctypes.byref(lob), N, seed, frames, None,
                                                      nirc._ptr(tl), nirc._ptr(c), None, nirc._stream()), "estimate")
        else:
            nirc._check(nirc.lib().tlmc_estimate(m.handle, dp.c(), nirc.ctypes.byref(lob), N, seed, frames, None,
                                                 nirc._ptr(tl), nirc._ptr(c), None, nirc._stream()), "estimate")
        st = nirc.tlmc_frame_stats(dp, lob, table, tl, c, fs=fs)
        q, tgt = nirc.tlmc_train_batch(dp, lob, 65536, seed + 7919, frames, 0)
        y = nirc.nirc_hash_infer(m, dp, q) if is_hash else nirc.nirc_infer(m, dp, q)
        flops = algorithmic_flops_hash(P, N) if is_hash else algorithmic_flops_estimate(P, N, 64)
        peak = PEAK_FP32_MFMA if name.endswith("fp32") else PEAK_BF16_MFMA
        out[name] = {"ms_estimate": ms, "queries_per_s": P * (N + 1) / (ms * 1e-3),
                     "tflops": flops / (ms * 1e-3) / 1e12, "mfma_frac": flops / (ms * 1e-3) / peak,
                     "mfma_peak_tflops": peak / 1e12, "flops_per_launch": flops, "ms_train_frame": t_train / frames,
                     "mrse": float(st[4].item()), "mrse_cache_only": float(st[5].item()),
                     "cache_rel_l2": float((y - tgt).norm() / tgt.norm()), "flags": m.read_flags(),
                     "cache_rel_l2_by_frame": curve}
    # the trained hash-grid cache in FP32, BF16 and FP16 over the direction counts of the
    # precision study: time, MFMA fraction and MRSE; 16-bit against FP32 on the same parameters
    hm = models["hash_grid_bf16"]
    wt = hm.get_weights()
    lob = nirc.lobes_struct(lobes_for(frames))
    sweep = []
    for Nq in (4, 16, 64):
        ref = None
        for pname, prec in (("fp32", 0), ("bf16", 1), ("fp16", 2)):
            mm = nirc.HashModel(wt, cfg=nirc.make_config(precision=prec), grid=grid, max_batch=0)
            out_t = torch.empty((P, 3), dtype=torch.float32, device="cuda")
            nirc.nirc_hash_estimate(mm, dp, lob, Nq, seed, frames, out=out_t)
            torch.cuda.synchronize()
            ev[0].record(stream)
            for _ in range(5):
                nirc.nirc_hash_estimate(mm, dp, lob, Nq, seed, frames, out=out_t)
            ev[1].record(stream)
            torch.cuda.synchronize()
            ms = ev[0].elapsed_time(ev[1]) / 5
            flops = algorithmic_flops_hash(P, Nq)
            mrse = float(nirc.tlmc_frame_stats(dp, lob, table, out_t, fs=fs)[4].item())
            peak = PEAK_FP32_MFMA if prec == 0 else PEAK_BF16_MFMA
            row = {"n_cache": Nq, "precision": pname, "ms_estimate": ms, "queries_per_s": P * (Nq + 1) / (ms * 1e-3),
                   "mfma_frac": flops / (ms * 1e-3) / peak, "mrse": mrse}
            if ref is None:
                ref = out_t.clone()
            else:
                row["rel_l2_vs_fp32"] = float((out_t - ref).norm() / ref.norm())
            sweep.append(row)
            del mm
    out["hash_precision_sweep"] = sweep
    # the same BF16 estimate with the points in a locality (Morton) order, as a renderer's
    # screen-space order would give them: the grid gather's cache lines are shared by neighbours
    if pts_host is not None:
        dpm = nirc.Points.from_workload(pts_host.subset(wl.morton_order(pts_host)))
        out_m = torch.empty((P, 3), dtype=torch.float32, device="cuda")
        nirc.nirc_hash_estimate(hm, dpm, lob, N, seed, frames, out=out_m)
        torch.cuda.synchronize()
        ev[0].record(stream)
        for _ in range(reps):
            nirc.nirc_hash_estimate(hm, dpm, lob, N, seed, frames, out=out_m)
        ev[1].record(stream)
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1]) / reps
        flops = algorithmic_flops_hash(P, N)
        out["hash_grid_bf16_locality_order"] = {
            "ms_estimate": ms, "queries_per_s": P * (N + 1) / (ms * 1e-3), "mfma_frac": flops / (ms * 1e-3) / PEAK_BF16_MFMA,
            "mrse": float(nirc.tlmc_frame_stats(dpm, lob, table, out_m, fs=fs)[4].item())}
        del dpm
    out["frames"] = frames
    out["grid_gather_bytes_per_point"] = 12 * 8 * 8
    return out


def ablation(nirc, w0, dp, lobes_packed, P, N, seed, reps=5, precision=1):
    """The paper's inference-pipeline comparison on this hardware: the estimate with its fusions
    undone (tlmc_estimate_unfused stage 0: every query's encoded inputs through memory; 1: the
    surface encoding shared per point; 2: the direction encoding inside the network kernel; 3:
    the fused estimator with per-point sums on chip), BF16, timed by HIP events."""
    import torch
    m = nirc.Model(w0, cfg=nirc.make_config(precision=precision), max_batch=0)
    lob = nirc.lobes_struct(lobes_packed)
    out = torch.empty((P, 3), dtype=torch.float32, device="cuda")
    Q = P * (N + 1)
    tiles, groups = (Q + 15) // 16, (P + 15) // 16
    # bytes each stage moves through HBM by design (points and outputs aside): operands written
    # and read back, per-query predictions written and read back
    traffic = {0: 2 * tiles * 6 * 1024 + 2 * Q * 12, 1: 2 * tiles * 2 * 1024 + 2 * groups * 4 * 1024 + 2 * Q * 12,
               2: 2 * groups * 4 * 1024 + 2 * Q * 12, 3: 0}
    rows = {}
    for stage in range(4):
        ws_bytes = nirc.tlmc_unfused_workspace_bytes(P, N, stage)
        ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device="cuda")
        run = lambda: nirc.tlmc_estimate_unfused(m, dp, lob, N, seed, 0, stage, workspace=ws, out=out)
        run()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        e[0].record()
        for _ in range(reps):
            run()
        e[1].record()
        torch.cuda.synchronize()
        ms = e[0].elapsed_time(e[1]) / reps
        rows[str(stage)] = {"ms_estimate": ms, "queries_per_s": Q / (ms * 1e-3), "workspace_bytes": ws_bytes,
                            "intermediate_hbm_bytes": traffic[stage]}
        del ws
    t0 = rows["0"]["ms_estimate"]
    for r in rows.values():
        r["speedup_vs_stage0"] = t0 / r["ms_estimate"]
    return {"points": P, "n_cache": N, "precision": "bf16" if precision == 1 else "fp16",
            "stages": {"0": "every query's encoded inputs written to and read from HBM, outputs per query, "
                            "separate reduction",
                       "1": "+ surface encoding once per point, shared by its N+1 queries",
                       "2": "+ direction sampling and encoding inside the network kernel",
                       "3": "+ surface projection once per point and per-point sums on chip (fused)"},
            "rows": rows,
            "paper_context": "1.74x / 2.62x / 3.64x over its fully-fused baseline (RTX 3080, hash + SH input)"}


def serving_run(seconds, budget_frac=0.4):
    """16 render streams (resolutions 360p..4K, N in {4, 8, 32}, width-64 BF16 caches with their
    own Adam state and training workspace), Poisson arrivals at 240 frames/s, admission by an HBM
    budget of `budget_frac` of what all streams would hold at once, continuous batching of each
    mix's estimate and training into one replayed graph, 4 training steps of 65,536 per frame."""
    import numpy as np
    from paper_2412_04634_amd import serve
    st, sch, ex = serve.serve_run(seed=5, n_streams=16, rate_hz=240.0, duration_s=seconds, precision=1,
                                  budget_bytes=budget_frac)
    st["budget_fraction"] = budget_frac
    st["mean_train_batch"] = float(np.mean(sch.batch_sizes))
    import torch
    nirc = ex.nirc
    specs = serve.make_stream_specs(5, 16)
    # the same frames run stream by stream: one frame of each stream alone (estimate + its
    # training steps) timed on the GPU, summed over the frames each stream received
    alone_ms = alone_frame_ms(nirc, ex, specs)
    counts = collections.Counter(f.sid for f in sch.done)
    serial_s = sum(alone_ms[sid] * n for sid, n in counts.items()) * 1e-3
    st["stream_by_stream"] = {"gpu_s": serial_s, "queries_per_s": st["queries"] / serial_s,
                              "frame_ms_by_stream": {str(k): v for k, v in sorted(alone_ms.items())}}
    # the same streams one frame each: one batched launch vs one launch per stream (GPU time)
    st["one_frame_per_stream"] = batched_vs_separate(nirc, ex, specs)
    # small frames (16 streams of 640 x 360, N = 4), where one launch per stream leaves the GPU
    # partly idle
    small = [serve.StreamSpec(100 + i, 640, 360, 4, 5000 + i, 5500) for i in range(16)]
    st["small_frames_16x360p_n4"] = batched_vs_separate(nirc, ex, small)
    return st


def alone_frame_ms(nirc, ex, specs, reps=3):
    """GPU time of one frame of each stream on its own: tlmc_estimate, then nirc_train_frame."""
    import torch
    ex.prepare(specs)
    out = {}
    for s in specs:
        if s.sid not in ex.streams:
            ex.admit(s)
        x = ex.streams[s.sid]
        lob = x["lobes"].packed()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]

        def one():
            nirc.tlmc_estimate(x["model"], x["points"], lob, s.n_cache, s.seed, 0, out=x["out"])
            nirc.nirc_train_frame(x["model"], x["points"], lob, ex.train_batch, ex.train_steps, s.seed, 0)
        one()
        torch.cuda.synchronize()
        e[0].record()
        for _ in range(reps):
            one()
        e[1].record()
        torch.cuda.synchronize()
        out[s.sid] = e[0].elapsed_time(e[1]) / reps
        ex.release(s.sid)
    return out


def batched_vs_separate(nirc, ex, specs, reps=5):
    """One frame of each stream: one batched persistent launch against one tlmc_estimate launch
    per stream (GPU time per round, average of `reps`)."""
    import torch
    ex.prepare(specs)
    for s in specs:
        if s.sid not in ex.streams:
            ex.admit(s)
    reqs = []
    for s in specs:
        x = ex.streams[s.sid]
        reqs.append(dict(model=x["model"], points=x["points"], lobes=x["lobes"].packed(), n_cache=s.n_cache,
                         seed=s.seed, frame=0, out_tl=x["out"]))
    b = nirc.Batch()
    b.set(reqs)
    b.launch()
    for r in reqs:
        nirc.tlmc_estimate(r["model"], r["points"], r["lobes"], r["n_cache"], r["seed"], 0, out=r["out_tl"])
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    torch.cuda.synchronize()
    e[0].record()
    for _ in range(reps):
        b.launch()
    e[1].record()
    for _ in range(reps):
        for r in reqs:
            nirc.tlmc_estimate(r["model"], r["points"], r["lobes"], r["n_cache"], r["seed"], 0, out=r["out_tl"])
    e[2].record()
    torch.cuda.synchronize()
    q = sum(s.points * (s.n_cache + 1) for s in specs)
    return {"queries": q, "batched_ms": e[0].elapsed_time(e[1]) / reps,
            "separate_launches_ms": e[1].elapsed_time(e[2]) / reps}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="1080p_n16")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision-compare", action="store_true")
    ap.add_argument("--train-only", choices=["fp32", "bf16", "hash-bf16", "hash-fp32"], default=None,
                    help="only time training frames (S steps of B samples) of this model")
    ap.add_argument("--estimate-only", choices=["fp32", "bf16", "fp16", "hash-bf16"], default=None,
                    help="time only tlmc_estimate at this precision (for profiling runs)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving leg (16 streams)")
    ap.add_argument("--ablation", action="store_true", help="add the unfused-pipeline comparison to the bench line")
    ap.add_argument("--ablation-only", action="store_true", help="only the unfused-pipeline comparison")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="duration of the multi-stream serving run (0 to skip)")
    ap.add_argument("--precision-form", action="store_true",
                    help="also run the N x width x precision matrix of estimates")
    ap.add_argument("--visibility", action="store_true",
                    help="visibility cache against a radiance cache on the occluded scene (100 frames each)")
    ap.add_argument("--loss-variants", action="store_true",
                    help="train a cache with each loss of the optimisation section (100 frames) and compare")
    ap.add_argument("--hash-grid", action="store_true",
                    help="also run the hash-grid / spherical-harmonics cache input against the frequency input")
    ap.add_argument("--train-convergence", action="store_true",
                    help="also run 300 frames of training only at batches 2^16, 2^18, 2^20")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="first run a plain device copy of this size (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; the hot path has no "
                                   "multi-GPU mode (--gpus must be 1)"}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2412_04634_amd import nirc, workload as wl

    cfgw = wl.WORKLOADS[args.workload]
    P, N, W, seed = cfgw["points"], cfgw["n_cache"], cfgw["width"], cfgw["seed"]
    B, S = cfgw["train_batch"], cfgw["train_steps"]
    dev = "cuda"
    torch.cuda.set_device(0)

    if args.serve_only:
        print(json.dumps({"serving": serving_run(args.serve_seconds)}), flush=True)
        return
    if args.ablation_only:
        pts = wl.make_points(seed, P)
        print(json.dumps({"ablation": ablation(nirc, wl.make_weights(seed, W), nirc.Points.from_workload(pts),
                                               wl.make_lobes(seed).packed(), P, N, seed, reps=args.steps)}),
              flush=True)
        return

    if args.copy_calibration > 0:
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.rand(n, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    scene = wl.make_scene(seed, P)
    w0 = wl.make_weights(seed, W)
    base_lobes = scene.lobes
    dp = nirc.Points.from_workload(scene.points)
    model = nirc.Model(w0, max_batch=B)
    lobes_frames = {}

    def lobes_for(f):
        if f not in lobes_frames:
            lobes_frames[f] = base_lobes.rotated(f).packed()
        return lobes_frames[f]

    if args.train_only:
        if args.train_only.startswith("hash-"):
            grid = nirc.make_hash_grid()
            m = nirc.HashModel(wl.make_hash_weights(seed, 64, 2 * nirc.nirc_hash_entries(grid)),
                               cfg=nirc.make_config(precision=1 if args.train_only == "hash-bf16" else 0), grid=grid,
                               max_batch=B)

            def train(f):
                nirc.nirc_hash_train_frame(m, dp, nirc.lobes_struct(lobes_for(f)), B, S, seed, f)
        else:
            m = nirc.Model(w0, cfg=nirc.make_config(precision={"fp32": 0, "bf16": 1}[args.train_only]), max_batch=B)

            def train(f):
                nirc.nirc_train_frame(m, dp, nirc.lobes_struct(lobes_for(f)), B, S, seed, f)
        for f in range(args.warmup):
            train(f)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(torch.cuda.current_stream())
        for f in range(args.steps):
            train(args.warmup + f)
        ev[1].record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        print(json.dumps({"train_only": args.train_only, "ms_train_frame": ev[0].elapsed_time(ev[1]) / args.steps,
                          "flags": m.read_flags()}), flush=True)
        return

    if args.estimate_only:
        lob = nirc.lobes_struct(lobes_for(0))
        out = torch.empty((P, 3), dtype=torch.float32, device=dev)
        if args.estimate_only == "hash-bf16":
            grid = nirc.make_hash_grid()
            m = nirc.HashModel(wl.make_hash_weights(seed, 64, 2 * nirc.nirc_hash_entries(grid)),
                               cfg=nirc.make_config(precision=1), grid=grid, max_batch=0)
            est = lambda: nirc.nirc_hash_estimate(m, dp, lob, N, seed, 0, out=out)
            flops = algorithmic_flops_hash(P, N)
        else:
            prec = {"fp32": 0, "bf16": 1, "fp16": 2}[args.estimate_only]
            m = nirc.Model(w0, cfg=nirc.make_config(precision=prec), max_batch=0)
            est = lambda: nirc.tlmc_estimate(m, dp, lob, N, seed, 0, out=out)
            flops = algorithmic_flops_estimate(P, N, W)
        for _ in range(args.warmup):
            est()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        torch.cuda.synchronize()
        ev[0].record(torch.cuda.current_stream())
        for _ in range(args.steps):
            est()
        ev[1].record(torch.cuda.current_stream())
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) * 1e-3 / args.steps
        print(json.dumps({"estimate_only": args.estimate_only, "ms_estimate": t * 1e3,
                          "tflops": flops / t / 1e12}), flush=True)
        return

    table = nirc.tlmc_reference_table(lobes_for(0))
    fs = nirc.FrameStats()
    out_tl = torch.empty((P, 3), dtype=torch.float32, device=dev)
    out_c = torch.empty_like(out_tl)
    out_r = torch.empty_like(out_tl)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    mrse_hist = []
    stream = torch.cuda.current_stream()

    def frame(f, ev=None):
        lob = nirc.lobes_struct(lobes_for(f))
        if ev is not None:
            ev[0].record(stream)
        nirc._check(nirc.lib().tlmc_estimate(model.handle, dp.c(), nirc.ctypes.byref(lob), N, seed, f, None,
                                             nirc._ptr(out_tl), nirc._ptr(out_c), nirc._ptr(out_r), nirc._stream()),
                    "tlmc_estimate")
        if ev is not None:
            ev[1].record(stream)
        st = nirc.tlmc_frame_stats(dp, lob, table, out_tl, out_c, out_r, fs=fs)
        if ev is not None:
            ev[2].record(stream)
        nirc.nirc_train_frame(model, dp, lob, B, S, seed, f, loss)
        if ev is not None:
            ev[3].record(stream)
        return st

    for f in range(args.warmup):
        frame(f)
    torch.cuda.synchronize()

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(args.steps)]
    stats = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        stats.append(frame(args.warmup + i, evs[i]).clone())
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    t_est = [e[0].elapsed_time(e[1]) * 1e-3 for e in evs]
    t_stats = [e[1].elapsed_time(e[2]) * 1e-3 for e in evs]
    t_train = [e[2].elapsed_time(e[3]) * 1e-3 for e in evs]
    t_frame = np.sort([e[0].elapsed_time(e[3]) for e in evs])
    mrse = [float(s[4].item()) for s in stats]
    # relative residual variance V_rel(F_r) per frame (mean F_r^2 / (F^2 + eps): the residual's
    # relative second moment, its variance once the cache integrates to F), smoothed over frames
    # with an exponential moving average of weight 0.95
    v_rel_ema = None
    for st_f in stats:
        v = float(st_f[6].item())
        v_rel_ema = v if v_rel_ema is None else 0.95 * v_rel_ema + 0.05 * v
    ms_frame = elapsed / args.steps * 1e3
    queries = P * (N + 1)
    value = queries * args.steps / elapsed
    t_est_avg = sum(t_est) / len(t_est)
    flops = algorithmic_flops_estimate(P, N, W)
    achieved = flops / t_est_avg

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "queries/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_frame,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"dynamic lobe scene, {P} shading points (1920x1080), N={N} cache + 1 residual, "
                               f"MLP 4x{W} ReLU, {S} Adam steps of {B} samples per frame",
                   "points": P, "n_cache": N, "width": W, "train_batch": B, "train_steps_per_frame": S,
                   "precision": "fp32"},
        "roofline": {"bound": "mfma", "kernel": "k_tlmc_f32", "achieved": achieved / 1e12,
                     "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_MFMA,
                     "traffic": TRAFFIC_K_TLMC_F32 if cfgw is wl.WORKLOADS["1080p_n16"] else None,
                     "traffic_unit": "bytes per launch", "flops_per_launch": flops,
                     "avg_launch_ms": t_est_avg * 1e3},
        "estimate_queries_per_s": queries / t_est_avg,
        "ms_estimate": t_est_avg * 1e3,
        "ms_frame_stats": sum(t_stats) / len(t_stats) * 1e3,
        "ms_train": sum(t_train) / len(t_train) * 1e3,
        "ms_frame_gpu_p50": float(np.percentile(t_frame, 50)),
        "ms_frame_gpu_p99": float(np.percentile(t_frame, 99)),
        "train_samples_per_s": S * B / (sum(t_train) / len(t_train)),
        "train_tflops": algorithmic_flops_train(B, W) * S / (sum(t_train) / len(t_train)) / 1e12,
        "mrse_first_last": [mrse[0], mrse[-1]],
        "v_rel_residual_ema": v_rel_ema,
        "final_loss": float(loss.item()),
    }
    probe = mfma_probe(nirc)
    result["mfma_probe"] = probe
    result["roofline"]["peak_measured"] = probe["fp32"]["tflops"]
    result["roofline"]["frac_measured"] = achieved / 1e12 / probe["fp32"]["tflops"]
    if result["roofline"]["traffic"] is not None:   # the HBM side of the same launch (far from its bound)
        result["roofline"]["hbm_gbps"] = result["roofline"]["traffic"] / t_est_avg / 1e9
        result["roofline"]["hbm_frac"] = result["roofline"]["traffic"] / t_est_avg / PEAK_HBM
    if not args.no_precision_compare:
        result["precision_compare"] = precision_compare(nirc, model, dp, lobes_for, table, fs, P, N, W, seed,
                                                        args.warmup + args.steps, args.steps, B, S)
        for name, v in result["precision_compare"].items():
            v["roofline"]["peak_measured"] = probe[name]["tflops"]
            v["roofline"]["frac_measured"] = v["roofline"]["achieved"] / probe[name]["tflops"]
        result["biased_bth"] = biased_compare(nirc, model, dp, lobes_for, table, fs, P, N, seed,
                                              args.warmup + args.steps, min(args.steps, 20))
        result["precision_trained"] = precision_trained(nirc, w0, dp, lobes_for, table, fs, P, N, seed, 100, B, S)
    if args.precision_form:
        result["precision_form"] = precision_form(nirc, model.get_weights(), dp, lobes_for(args.warmup + args.steps),
                                                  table, fs, P, seed, args.warmup + args.steps)
    if args.visibility:
        result["visibility"] = visibility_compare(nirc, w0, dp, lobes_for, P, N, seed, 100, B, S)
    if args.hash_grid:
        result["hash_grid"] = hash_grid_compare(nirc, w0, dp, lobes_for, table, fs, P, N, seed, 100, B, S,
                                                pts_host=scene.points)
    if args.loss_variants:
        result["loss_variants"] = loss_variants(nirc, w0, dp, lobes_for, table, fs, P, N, seed, 100, B, S)
    if args.train_convergence:
        result["train_convergence"] = {p: train_convergence(nirc, dp, lobes_for, W, seed, precision=i)
                                       for p, i in (("fp32", 0), ("bf16", 1))}
    if args.ablation:
        result["ablation"] = ablation(nirc, w0, dp, lobes_for(0), P, N, seed)
    if args.serve_seconds > 0:
        result["serving"] = serving_run(args.serve_seconds)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(scene.points, lobes_for, w0, W, N, B, S)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
