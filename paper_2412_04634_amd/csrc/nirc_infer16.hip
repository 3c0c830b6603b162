// BF16 / FP16 inference kernels: per-query inference and the fused two-level estimator with
// 16-bit MFMA operands and FP32 accumulation (master weights stay FP32; a 16-bit packed copy is
// refreshed after every Adam step).
#include "nirc_hash.hpp"

namespace nirc {

// packed16[e] = 16-bit(master[source(e)]) (round to nearest even), zero padding elsewhere.
// After an Adam step (step != NULL) thread 0 also commits the step or records its skip.
// (W is a template parameter so that the section search folds to constants.)
template <int PREC, int W>
__device__ __forceinline__ void pack16_elem(uint16_t *packed, const float *master, int total, int64_t *step,
                                            uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good,
                                            int e) {
    if (e < total) {
        const int64_t s = h16_packed_source(W, e);
        const float v = s >= 0 ? master[s] * h16_packed_scale(W, e) : 0.0f;
        packed[e] = (uint16_t)(pack2<PREC>(v, 0.0f) & 0xFFFFu);
    }
    if (step && e == 0) commit_step(step, flags, bad, dyn_scale, good);
}

template <int PREC, int W>
__global__ void k_pack16(uint16_t *packed, const float *master, int total, int64_t *step, uint32_t *flags,
                         uint32_t *bad, float *dyn_scale, uint32_t *good) {
    pack16_elem<PREC, W>(packed, master, total, step, flags, bad, dyn_scale, good, blockIdx.x * blockDim.x + threadIdx.x);
}

// Adam on the FP32 master weights with the 16-bit copy refreshed in the same pass: thread i
// updates parameter i (the arithmetic of adam_elem) and stores it, scaled, into every packed
// element that holds it (h16_packed_targets); a skipped step (`bad` set) changes nothing.  The
// last workgroup to finish (counted in `done`) commits the step as pack16_elem does: every other
// workgroup has read `step` and `bad` before it counted itself.
template <int PREC, int W>
__device__ __forceinline__ void adam_pack16_block(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                                  const float *__restrict__ grad, int64_t *step, uint32_t *flags,
                                                  uint32_t *bad, float *dyn_scale, uint32_t *good, uint32_t *done,
                                                  uint16_t *__restrict__ packed, float lr, float b1, float b2,
                                                  float eps, int blk, int nblk) {
    constexpr int64_t np = n_params(W);
    const int64_t i = (int64_t)blk * blockDim.x + threadIdx.x;
    if (i < np && *bad == 0u) {
        const float t = (float)(*step + 1);
        const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
        float mi = m[i], vi = v[i];
        const float wi = adam_update(w[i], mi, vi, grad[i], c1, c2, lr, b1, b2, eps);
        m[i] = mi;
        v[i] = vi;
        w[i] = wi;
        int e[6];
        float sc[6];
        const int n = h16_packed_targets(W, i, e, sc);
        for (int k = 0; k < n; ++k) packed[e[k]] = (uint16_t)(pack2<PREC>(wi * sc[k], 0.0f) & 0xFFFFu);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(done, 1u) == (uint32_t)nblk - 1u) {
            __threadfence();
            commit_step(step, flags, bad, dyn_scale, good);
            *done = 0u;
        }
    }
}

template <int PREC, int W>
__global__ __launch_bounds__(kAdamThreads) void k_adam_pack16(float *w, float *m, float *v, const float *grad, int64_t *step,
                                                     uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good,
                                                     uint32_t *done, uint16_t *packed, float lr, float b1, float b2,
                                                     float eps) {
    adam_pack16_block<PREC, W>(w, m, v, grad, step, flags, bad, dyn_scale, good, done, packed, lr, b1, b2, eps,
                               blockIdx.x, gridDim.x);
}

// Adam + repack + commit of every request of a training work list (request blockIdx.y).
template <int PREC, int W>
__global__ __launch_bounds__(kAdamThreads) void k_adam_pack16_multi(const TrainDesc *__restrict__ desc) {
    if ((int)blockIdx.y >= desc->n) return;
    const TrainReq &t = desc->req[blockIdx.y];
    adam_pack16_block<PREC, W>(t.master, t.m, t.v, t.grad, t.step, t.flags, t.bad, t.dyn_scale, t.good_steps,
                               t.done, const_cast<uint16_t *>(t.packed16), t.lr, t.b1, t.b2, t.eps, blockIdx.x,
                               gridDim.x);
}

hipError_t launch_adam_pack16(int W, int prec, float *w, float *m, float *v, const float *grad, int64_t *step,
                              uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good, uint32_t *done,
                              uint16_t *packed, float lr, float b1, float b2, float eps, hipStream_t s) {
    const dim3 grid((unsigned)((n_params(W) + kAdamThreads - 1) / kAdamThreads)), block(kAdamThreads);
    if (W == 64 && prec == NIRC_BF16)
        hipLaunchKernelGGL((k_adam_pack16<NIRC_BF16, 64>), grid, block, 0, s, w, m, v, grad, step, flags, bad, dyn_scale,
                           good, done, packed, lr, b1, b2, eps);
    else if (W == 64)
        hipLaunchKernelGGL((k_adam_pack16<NIRC_FP16, 64>), grid, block, 0, s, w, m, v, grad, step, flags, bad, dyn_scale,
                           good, done, packed, lr, b1, b2, eps);
    else if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_adam_pack16<NIRC_BF16, 128>), grid, block, 0, s, w, m, v, grad, step, flags, bad,
                           dyn_scale, good, done, packed, lr, b1, b2, eps);
    else
        hipLaunchKernelGGL((k_adam_pack16<NIRC_FP16, 128>), grid, block, 0, s, w, m, v, grad, step, flags, bad,
                           dyn_scale, good, done, packed, lr, b1, b2, eps);
    return hipGetLastError();
}

hipError_t launch_adam_pack16_multi(const TrainDesc *desc, int W, int prec, hipStream_t s) {
    if (W != 64) return hipErrorInvalidValue;
    const dim3 grid((unsigned)((n_params(64) + kAdamThreads - 1) / kAdamThreads), kBatchMaxRequests), block(kAdamThreads);
    if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_adam_pack16_multi<NIRC_BF16, 64>), grid, block, 0, s, desc);
    else
        hipLaunchKernelGGL((k_adam_pack16_multi<NIRC_FP16, 64>), grid, block, 0, s, desc);
    return hipGetLastError();
}

template <int W>
struct Infer16Lds {
    static constexpr int kWeights = H16Layout{W}.offset(SEC_T0) - H16Layout{W}.offset(SEC_D);   // elements
};

// Per-query inference: 16 queries per wave per iteration, all 160 features per query.
template <int W, int PREC, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_infer_h16(Points pts, Queries q, const uint16_t *__restrict__ packed,
                                                          float *__restrict__ rgb, int sig) {
    constexpr H16Layout L{W};
    constexpr int MT = W / 16, KB = W / 32;
    constexpr bool kLds = lds_weights(W);
    constexpr int NW = kLds ? Infer16Lds<W>::kWeights : 8;
    __shared__ u32x4 smem4[NW / 8];
    if constexpr (kLds) {
        const u32x4 *src = (const u32x4 *)(packed + L.offset(SEC_D));
        for (int i = threadIdx.x; i < NW / 8; i += WAVES * 64) smem4[i] = src[i];
        __syncthreads();
    }
    const uint16_t *gS = packed + L.offset(SEC_S);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t Q = q.count;
    const int64_t n_tiles = (Q + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * WAVES + wave; tile < n_tiles; tile += (int64_t)gridDim.x * WAVES) {
        const uint16_t *sD = kLds ? (const uint16_t *)smem4 : opaque(packed) + L.offset(SEC_D);
        const uint16_t *sH = sD + L.size(SEC_D);
        const uint16_t *sO = sH + 3 * L.size(SEC_H0);
        const int64_t qi = min((tile << 4) + col, Q - 1);
        const int64_t p = query_point(q, pts, qi);
        const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
        f32x4 h[1][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) h[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        layer1_surface16<W, PREC>(h[0], opaque(gS), xs, lane, g);
        u32x4 bd[1][2];
        direction_operands<PREC>(q.wx[qi], q.wy[qi], q.wz[qi], g, bd[0][0], bd[0][1]);
        u32x4 hb[1][KB];
        u32x4 aout[4 * KB];
        if constexpr (kLds) {
            u32x4 dfrag[W / 8];
            load_dir_fragments<W>(dfrag, sD, lane);
            mlp16<W, PREC, 1>(h, hb, bd, dfrag, sH, sO + L.size(SEC_O), lane, aout);
        } else {
            mlp16_wide<W, PREC, 1>(h, hb, bd, sD, sH, sO + L.size(SEC_O), lane, aout);
        }
        // lane (g, c < 3) holds channel c of queries 4g + i of this tile
        const f32x4 z = output16_packed<W, PREC, 1>(hb, aout);
        if (col < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t qo = (tile << 4) + 4 * g + i;
                if (qo < Q) rgb[3 * qo + col] = sig ? 1.0f / (1.0f + __expf(-z[i])) : __expf(z[i]);
            }
        }
    }
}

// Per-wave scratch of the estimator's point group (LDS).
struct GroupSlab {
    float *hs;     // [16 points][W] surface projection
    float *db;     // [3][kDirSlots] staged directions
    float *psum;   // [16 points][4] cache-level sums
    float *yres;   // [16 points][4] residual-direction predictions
    float *qbuf;   // [16 queries][4] one tile's predictions (general N only)
    float *nrm;    // [3][16] normals of the group's points
    u32x4 *fa;     // [4 tiles][4 lane groups][16 queries] direction features, first K-block
    uint2 *fb;     // [4 tiles][4 lane groups][16 queries] direction features, second K-block
};

// Direction features of a 4-tile pass are staged in the slab at width 64 only; wider models
// compute each tile's direction operands in the lanes that use them (and give the room to their
// hidden-layer weights).
template <int W>
struct Tlmc16Lds {
    static constexpr int kSlab = TlmcLds<W>::kSlab + 48 + (lds_weights(W) ? 4 * 64 * 4 + 4 * 64 * 2 : 0);   // floats
};

// T consecutive query tiles (first tile T0, staged directions from batch slot s0) of the
// current point group through the 16-bit chain.  The output layer of all T tiles lands in one
// accumulator (tile tt in columns 3tt..3tt+2), so the exponential and the per-point sums are
// done once per pass: a lane holds 4 consecutive queries of one tile and channel.
// OCC: the occluded-scene variants (visibility cache, radiance cache of the occluded scene),
// selected at run time by `mode`; the radiance cache of the plain scene compiles without them.
// ENC 1: the hash-grid model's direction input (25 spherical harmonics, one K-block).
// HL: the hidden layers' fragments are in LDS (sH) while the direction and output sections stay
// in global memory (widths above 64).
// N16: n_cache is a multiple of 16 (the per-point sums take only the first of the three paths
// below; compiling the others out measured 2.4 % shorter estimates at N = 16).
template <int W, int PREC, int T, bool OCC, int ENC = 0, bool HL = false, bool N16 = false>
__device__ __forceinline__ void tlmc_tiles_h16(int T0, int s0, int n_cache, DivN dn, const GroupSlab &gs,
                                               const uint16_t *sD, const uint16_t *sH, const uint16_t *sOS,
                                               const u32x4 (&dfrag)[W / 8], int lane, int g, int col, float &rdx,
                                               float &rdy, float &rdz, const Points &pts, int64_t p0, int mode,
                                               const nirc_lobes &lobes) {
    constexpr int MT = W / 16, KB = W / 32;
    f32x4 h[T][MT];
    u32x4 bd[T][2];
    // hidden layers in LDS: the direction layer's fragments come from global memory, requested
    // before the pass's direction operands are built so that their latency sits under that work
    u32x4 dl2[HL ? W / 8 : 1];
    if constexpr (HL) load_dir_fragments<W, 2>(dl2, opaque(sD), lane);
    if constexpr (T == 4 && lds_weights(W)) {
        // a full pass: lane 16 tt + c encodes query c of tile tt once (all frequencies, by angle
        // doubling) into LDS, where every lane group picks up its part of the B operands
        const int q = 16 * s0 + lane;
        const int e0 = 64 * (lane >> 4) + (lane & 15);   // entry (tile lane / 16, group 0, query lane % 16)
        wave_lds_order();   // after the previous pass's reads of fa / fb
        if constexpr (ENC == 1)
            sh_features16<PREC>(gs.db[q], gs.db[kDirSlots + q], gs.db[2 * kDirSlots + q], gs.fa + e0, 16);
        else
            dir_features16<PREC>(gs.db[q], gs.db[kDirSlots + q], gs.db[2 * kDirSlots + q], gs.fa + e0, gs.fb + e0,
                                 16);
        wave_lds_order();
    }
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const int Tt = T0 + tt;
        const int qi = 16 * (s0 + tt) + col;
        if (Tt == n_cache) {   // residual tile: keep this column's direction for the final combine
            rdx = gs.db[qi];
            rdy = gs.db[kDirSlots + qi];
            rdz = gs.db[2 * kDirSlots + qi];
        }
        // the point of this column's query; with N a multiple of 16 a cache tile holds one point
        // (a wave-uniform row of the slab)
        const int j = (Tt < n_cache) ? (int)div_n((uint32_t)(N16 ? 16 * Tt : 16 * Tt + col), dn) : col;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) h[tt][mt] = *(const f32x4 *)(gs.hs + j * W + 16 * mt + 4 * g);
        if constexpr (T == 4 && lds_weights(W)) {
            const int e = (tt * 4 + g) * 16 + col;
            bd[tt][0] = gs.fa[e];
            if constexpr (ENC == 1) {
                bd[tt][1] = u32x4{0u, 0u, 0u, 0u};
            } else {
                const uint2 b = gs.fb[e];
                bd[tt][1] = u32x4{b.x, b.y, 0u, 0u};
            }
        } else if constexpr (ENC == 1) {
            bd[tt][0] = sh_operand<PREC>(gs.db[qi], gs.db[kDirSlots + qi], gs.db[2 * kDirSlots + qi], g);
            bd[tt][1] = u32x4{0u, 0u, 0u, 0u};
        } else {
            direction_operands<PREC>(gs.db[qi], gs.db[kDirSlots + qi], gs.db[2 * kDirSlots + qi], g, bd[tt][0],
                                     bd[tt][1]);
        }
    }
    u32x4 hb[T][KB];
    u32x4 aout[4 * KB];
    if constexpr (lds_weights(W)) {
        mlp16<W, PREC, T, ENC == 1 ? 1 : 2>(h, hb, bd, dfrag, sH, sOS, lane, aout);
    } else {   // weights in global memory: keep their loads inside the pass
        if constexpr (HL)
            mlp16_hl<W, PREC, T>(h, hb, bd, dl2, sH, opaque(sOS), lane, aout);
        else
            mlp16_wide<W, PREC, T>(h, hb, bd, opaque(sD), opaque(sH), opaque(sOS), lane, aout);
    }
    const f32x4 z = output16_packed<W, PREC, T>(hb, aout);

    // lane (g, col): tile tt = col / 3, channel c = col % 3, queries 4g + i of that tile
    const int tt = col / 3, c = col - 3 * (col / 3);
    const bool valid = col < 3 * T;
    const int Tt = T0 + tt;
    const int q0 = 4 * g;   // first query (row) of this lane within its tile
    float e0, e1, e2, e3;
    if (OCC && mode == NIRC_OUTPUT_VISIBILITY) {
        // uniform: predicted visibility times channel c of the known radiance, for this lane's
        // four queries (their staged directions and their points' positions)
        const int ts = min(tt, T - 1);   // lanes past the pass's tiles compute an unused value
        const int Ts = T0 + ts;
        float ev[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int qi = 16 * (s0 + ts) + q0 + i;
            const int j = (Ts < n_cache) ? (int)div_n((uint32_t)(16 * Ts + q0 + i), dn) : q0 + i;
            const int64_t pj = min(p0 + j, pts.count - 1);
            const float Lc = field_channel(lobes, c, pts.px[pj], pts.py[pj], pts.pz[pj], gs.db[qi],
                                           gs.db[kDirSlots + qi], gs.db[2 * kDirSlots + qi]);
            ev[i] = Lc / (1.0f + __expf(-z[i]));
        }
        e0 = ev[0];
        e1 = ev[1];
        e2 = ev[2];
        e3 = ev[3];
    } else {
        e0 = __expf(z[0]);
        e1 = __expf(z[1]);
        e2 = __expf(z[2]);
        e3 = __expf(z[3]);
    }
    if (N16 || (n_cache & 15) == 0) {
        float sum = (e0 + e1) + (e2 + e3);
        sum += __shfl_xor(sum, 16);
        sum += __shfl_xor(sum, 32);
        // one point per tile, N / 16 consecutive tiles per point.  A pass of T = 2 or 4 tiles
        // starts at a tile index divisible by T, so its tiles of one point are neighbours in the
        // pass: fold them into the lane of the run's last tile (tile tt sits 3 columns after tile
        // tt - 1), which then adds to the point's sum; every storing lane has its own point.
        bool last = true;
        if constexpr (T >= 2) {
            const int tpp = n_cache >> 4;
            if (tpp >= 2) {
                sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0x113, 0xF,
                                                                           0xF, true));   // row_shr:3
                if (T == 4 && tpp >= 4)
                    sum += __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, sum), 0x116,
                                                                               0xF, 0xF, true));   // row_shr:6
                last = ((tt + 1) & (min(tpp, T) - 1)) == 0;
            }
        }
        if (valid && last && g == 0 && Tt < n_cache) gs.psum[div_n((uint32_t)(16 * Tt), dn) * 4 + c] += sum;
    } else if constexpr (!N16) {
        if (n_cache <= 8 && (16 % n_cache) == 0) {
            // every point of a cache tile lies inside the tile: plain stores of complete sums
            if (valid && Tt < n_cache) {
                const int pbase = (int)div_n((uint32_t)(16 * Tt + q0), dn);   // point of this lane's first query
                if (n_cache == 1) {
                    gs.psum[(pbase + 0) * 4 + c] = e0;
                    gs.psum[(pbase + 1) * 4 + c] = e1;
                    gs.psum[(pbase + 2) * 4 + c] = e2;
                    gs.psum[(pbase + 3) * 4 + c] = e3;
                } else if (n_cache == 2) {
                    gs.psum[(pbase + 0) * 4 + c] = e0 + e1;
                    gs.psum[(pbase + 1) * 4 + c] = e2 + e3;
                } else if (n_cache == 4) {
                    gs.psum[pbase * 4 + c] = (e0 + e1) + (e2 + e3);
                }
            }
            if (n_cache == 8) {
                float sum = (e0 + e1) + (e2 + e3);
                sum += __shfl_xor(sum, 16);
                if (valid && Tt < n_cache && (g & 1) == 0) gs.psum[((16 * Tt + q0) / 8) * 4 + c] = sum;
            }
        } else {
            // any other N: tile by tile through a query buffer, one lane per channel summing in order
#pragma unroll
            for (int u = 0; u < T; ++u) {
                if (valid && tt == u) {
                    gs.qbuf[(q0 + 0) * 4 + c] = e0;
                    gs.qbuf[(q0 + 1) * 4 + c] = e1;
                    gs.qbuf[(q0 + 2) * 4 + c] = e2;
                    gs.qbuf[(q0 + 3) * 4 + c] = e3;
                }
                wave_sync();
                if (lane < 3 && T0 + u < n_cache) {
                    for (int q = 0; q < 16; ++q) {
                        const int pt = (int)div_n((uint32_t)(16 * (T0 + u) + q), dn);
                        gs.psum[pt * 4 + lane] += gs.qbuf[q * 4 + lane];
                    }
                }
                wave_sync();
            }
        }
    }
    // residual tile: predictions at each point's residual direction (query j = point j)
    if (valid && Tt == n_cache) {
        gs.yres[(q0 + 0) * 4 + c] = e0;
        gs.yres[(q0 + 1) * 4 + c] = e1;
        gs.yres[(q0 + 2) * 4 + c] = e2;
        gs.yres[(q0 + 3) * 4 + c] = e3;
    }
}

// One point group (16 points from p0) of the fused estimator: surface projection once per point
// into the slab, then the N + 1 query tiles in passes of 4 (and single-tile remainders), then the
// per-point combine and store.  Weights for the direction/hidden/output layers are in LDS; the
// surface columns are read from global memory (gS).
// ENC 1: the hash-grid model (surface part from the grid `slv`/`table` and phi, direction part
// from spherical harmonics).
template <int W, int PREC, int TP, bool OCC, int ENC = 0, bool HL = false, bool N16 = false>
__device__ __forceinline__ void tlmc_group_h16(const Points &pts, int64_t p0, int n_cache, DivN dn, uint32_t key0,
                                               uint32_t key1, uint32_t frame, int mode, const float *rrad,
                                               float *out_tl,
                                               float *out_c, float *out_r, const nirc_lobes &lobes, const uint16_t *gS,
                                               const uint16_t *sD, const uint16_t *sH, const uint16_t *sOS,
                                               const GroupSlab &gs, int lane, int g, int col,
                                               const HashLevel *slv = nullptr, uint32_t tmask = 0u,
                                               const float2 *table = nullptr, const float2 *fetched = nullptr,
                                               float2 (*prefetch)[24] = nullptr, int64_t prefetch_pc = 0) {
    constexpr int MT = W / 16;
    const int64_t P = pts.count;
    const int n_tiles = n_cache + 1;
    const int64_t pc = min(p0 + col, P - 1);
    const float xs[7] = {pts.px[pc], pts.py[pc], pts.pz[pc], pts.nx[pc], pts.ny[pc], pts.nz[pc], pts.rough[pc]};
    {
        f32x4 hsum[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) hsum[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        if constexpr (ENC == 1) {
            static_assert(W == 64, "the hash-grid model has width 64");
            u32x4 b0, b1;
            float v[6];
            // corner features fetched one group ahead by the caller
            hash_blend6(slv, xs[0], xs[1], xs[2], g, *(const float2(*)[24])fetched, v);
            hash_pack_surface<PREC>(xs, g, v, b0, b1);
            hash_layer1_surface<PREC>(hsum, opaque(gS), b0, b1, lane);
        } else {
            layer1_surface16<W, PREC>(hsum, opaque(gS), xs, lane, g);
        }
        wave_sync();   // the previous group's readers of the slab are done
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) *(f32x4 *)(gs.hs + col * W + 16 * mt + 4 * g) = hsum[mt];
        gs.psum[lane] = 0.0f;
        if (g < 3) gs.nrm[16 * g + col] = g == 0 ? xs[3] : g == 1 ? xs[4] : xs[5];   // normal of point col
        wave_sync();
    }
    float rdx = 0.f, rdy = 0.f, rdz = 0.f;
    u32x4 dfrag[W / 8];   // direction-layer fragments, resident across the group's passes
    if constexpr (lds_weights(W)) load_dir_fragments<W, ENC == 1 ? 1 : 2>(dfrag, sD, lane);
    for (int tb = 0; tb < n_tiles;) {
        const bool fold = n_tiles - tb == 9;   // last 8 cache tiles + the residual tile
        gen_dirs_batch_nrm<true>((uint32_t)p0, tb, n_cache, dn, key0, key1, frame, lane, gs.db, gs.nrm, fold);
        const int tend = fold ? n_tiles : min(tb + 8, n_tiles);
        if constexpr (ENC == 1) {
            // the next group's grid corners, fetched behind this group's last tiles (after the
            // last direction batch, whose point loads would otherwise wait for them)
            if (tend == n_tiles && prefetch)
                hash_fetch24(slv, tmask, table, pts.px[prefetch_pc], pts.py[prefetch_pc], pts.pz[prefetch_pc], g,
                             *prefetch);
        }
        int t = tb;
#pragma unroll 1
        for (; t + TP <= tend; t += TP)
            tlmc_tiles_h16<W, PREC, TP, OCC, ENC, HL, N16>(t, t - tb, n_cache, dn, gs, sD, sH, sOS, dfrag, lane, g, col, rdx, rdy,
                                                 rdz, pts, p0, mode, lobes);
#pragma unroll 1
        for (; t < tend; ++t)
            tlmc_tiles_h16<W, PREC, 1, OCC, ENC, HL, N16>(t, t - tb, n_cache, dn, gs, sD, sH, sOS, dfrag, lane, g, col, rdx, rdy,
                                                rdz, pts, p0, mode, lobes);
        tb = tend;
    }
    wave_sync();
    // residual sample: the caller's radiance (uniform branch), or the field: lane group g
    // evaluates lobe g at its column's point and residual direction, and the four lobes are
    // summed across the lane groups
    float Lr[3];
    if (rrad) {
        Lr[0] = rrad[3 * pc];
        Lr[1] = rrad[3 * pc + 1];
        Lr[2] = rrad[3 * pc + 2];
    } else {
        field_lobe(lobes, g, xs[0], xs[1], xs[2], rdx, rdy, rdz, Lr);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Lr[c] += __shfl_xor(Lr[c], 16);
            Lr[c] += __shfl_xor(Lr[c], 32);
        }
        if (OCC && mode != NIRC_OUTPUT_RADIANCE) {   // the occluded scene's residual sample V L
            const float V = visibility(lobes, xs[0], rdx, rdy, rdz);
            Lr[0] *= V;
            Lr[1] *= V;
            Lr[2] *= V;
        }
    }
    if (g == 0 && p0 + col < P) {
        const float inv_n = 1.0f / (float)n_cache;
        const float *ps = gs.psum + 4 * col, *yr = gs.yres + 4 * col;
        store_estimate(p0 + col, inv_n, ps[0], ps[1], ps[2], Lr[0] - yr[0], Lr[1] - yr[1], Lr[2] - yr[2], out_tl,
                       out_c, out_r);
    }
}

__device__ inline GroupSlab group_slab(float *base, int W) {
    GroupSlab gs;
    gs.hs = base;
    gs.db = gs.hs + 16 * W;
    gs.psum = gs.db + 3 * kDirSlots;
    gs.yres = gs.psum + 64;
    gs.qbuf = gs.yres + 64;
    gs.nrm = gs.qbuf + 64;
    gs.fa = (u32x4 *)(gs.nrm + 48);
    gs.fb = (uint2 *)(gs.fa + 4 * 64);
    return gs;
}

// Fused two-level estimator for one request: 16 points per wave at a time, grid-stride over
// point groups; weights staged once per workgroup.
template <int W, int PREC, int WAVES, bool OCC, bool N16>
__global__ __launch_bounds__(WAVES * 64) void k_tlmc_h16(Points pts, nirc_lobes lobes, const uint16_t *__restrict__ packed,
                                                         int n_cache, DivN dn, uint32_t key0, uint32_t key1,
                                                         uint32_t frame, int mode, const float *__restrict__ rrad,
                                                         float *__restrict__ out_tl, float *__restrict__ out_c,
                                                         float *__restrict__ out_r) {
    constexpr H16Layout L{W};
    constexpr bool kLds = lds_weights(W);
    constexpr int SLAB = Tlmc16Lds<W>::kSlab;                   // floats per wave
    // wider models: the hidden layers alone go to LDS when they fit beside the slabs
    constexpr int kHid = 3 * L.size(SEC_H0);                    // 16-bit elements
    constexpr bool kHidLds = !kLds && kHid * 2 + WAVES * SLAB * 4 + 1024 <= 160 * 1024;
    constexpr int NW = kLds ? Infer16Lds<W>::kWeights : kHidLds ? kHid : 8;   // 16-bit elements
    __shared__ u32x4 wsm[NW / 8];
    __shared__ f32x4 slab4[WAVES * SLAB / 4];
    __shared__ nirc_lobes s_lobes;
    {
        const u32x4 *src = (const u32x4 *)(packed + L.offset(kLds ? SEC_D : SEC_H0));
        if (kLds || kHidLds)
            for (int i = threadIdx.x; i < NW / 8; i += WAVES * 64) wsm[i] = src[i];
        if (threadIdx.x == 0) s_lobes = lobes;
    }
    __syncthreads();
    const uint16_t *sD = kLds ? (const uint16_t *)wsm : packed + L.offset(SEC_D);
    const uint16_t *sH = kHidLds ? (const uint16_t *)wsm : sD + L.size(SEC_D);
    const uint16_t *sOS = kLds ? sH + 3 * L.size(SEC_H0) + L.size(SEC_O) : packed + L.offset(SEC_OS);
    const uint16_t *gS = packed + L.offset(SEC_S);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const GroupSlab gs = group_slab((float *)slab4 + wave * SLAB, W);
    const int64_t n_groups = (pts.count + 15) >> 4;
    for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES)
        tlmc_group_h16<W, PREC, (W <= 64 || WAVES <= 4) ? 4 : 2, OCC, 0, kHidLds, N16>(
            pts, grp << 4, n_cache, dn, key0, key1, frame, mode, rrad, out_tl, out_c, out_r, s_lobes, gS, sD, sH, sOS,
            gs, lane, g, col);
}

// Continuous batching: a persistent grid walks a device work list of requests (each with its own
// model, points, field, N, seed and frame).  Work is cut into chunks of WAVES point groups of one
// request; a workgroup takes chunks in grid-stride order and re-stages weights and field in LDS
// only when the request changes.  The list lives in device memory, so a captured launch can be
// replayed with a different mix.
template <int W, int PREC, int WAVES, bool OCC>
__global__ __launch_bounds__(WAVES * 64) void k_tlmc_multi_h16(const BatchDesc *__restrict__ desc) {
    constexpr H16Layout L{W};
    constexpr int NW = Infer16Lds<W>::kWeights;
    constexpr int SLAB = Tlmc16Lds<W>::kSlab;
    __shared__ u32x4 wsm[NW / 8];
    __shared__ f32x4 slab4[WAVES * SLAB / 4];
    __shared__ BatchRequest s_req;
    const uint16_t *sD = (const uint16_t *)wsm;
    const uint16_t *sH = sD + L.size(SEC_D);
    const uint16_t *sOS = sH + 3 * L.size(SEC_H0) + L.size(SEC_O);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const GroupSlab gs = group_slab((float *)slab4 + wave * SLAB, W);
    const int n_req = desc->n_requests;
    const int total = desc->total_chunks;
    int cur = -1;
    for (int chunk = blockIdx.x; chunk < total; chunk += gridDim.x) {
        // request owning this chunk (uniform): last r with chunk_begin <= chunk
        int r = 0;
        for (int i = 1; i < n_req; ++i)
            if (desc->req[i].chunk_begin <= chunk) r = i;
        if (r != cur) {
            __syncthreads();   // every wave is done with the previous request's weights
            if (threadIdx.x == 0) s_req = desc->req[r];
            __syncthreads();
            const u32x4 *src = (const u32x4 *)((const uint16_t *)s_req.packed + L.offset(SEC_D));
            for (int i = threadIdx.x; i < NW / 8; i += WAVES * 64) wsm[i] = src[i];
            __syncthreads();
            cur = r;
        }
        const int64_t grp = (int64_t)(chunk - s_req.chunk_begin) * WAVES + wave;
        if (grp < (s_req.pts.count + 15) >> 4)
            tlmc_group_h16<W, PREC, 4, OCC>(s_req.pts, grp << 4, s_req.n_cache, s_req.dn, s_req.key0, s_req.key1, s_req.frame,
                                    __builtin_amdgcn_readfirstlane(s_req.mode), uniform_ptr(s_req.rrad), s_req.out_tl,
                                    s_req.out_c, s_req.out_r, s_req.lobes,
                                    (const uint16_t *)s_req.packed + L.offset(SEC_S), sD, sH, sOS, gs, lane, g, col);
    }
}

// ------------------------------------------------------------------------------------------



hipError_t launch_pack16(uint16_t *packed, const float *master, int W, int prec, hipStream_t s, int64_t *step,
                         uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good) {
    if (W != 64 && W != 128) return hipErrorInvalidValue;
    const int total = H16Layout{W}.total();
    const dim3 grid((total + 255) / 256), block(256);
    if (prec == NIRC_BF16 && W == 64)
        hipLaunchKernelGGL((k_pack16<NIRC_BF16, 64>), grid, block, 0, s, packed, master, total, step, flags, bad, dyn_scale, good);
    else if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_pack16<NIRC_BF16, 128>), grid, block, 0, s, packed, master, total, step, flags, bad, dyn_scale, good);
    else if (W == 64)
        hipLaunchKernelGGL((k_pack16<NIRC_FP16, 64>), grid, block, 0, s, packed, master, total, step, flags, bad, dyn_scale, good);
    else
        hipLaunchKernelGGL((k_pack16<NIRC_FP16, 128>), grid, block, 0, s, packed, master, total, step, flags, bad, dyn_scale, good);
    return hipGetLastError();
}

hipError_t launch_infer_h16(int W, int prec, const Points &pts, const Queries &q, const void *packed, float *rgb,
                            int sig, hipStream_t s) {
    constexpr int WAVES = 4;
    const unsigned grid = grid_for((q.count + 15) / 16, WAVES, 4 * kMaxResidentBlocks);
    const uint16_t *pk = (const uint16_t *)packed;
    if (W == 64 && prec == NIRC_BF16)
        hipLaunchKernelGGL((k_infer_h16<64, NIRC_BF16, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q, pk, rgb, sig);
    else if (W == 64)
        hipLaunchKernelGGL((k_infer_h16<64, NIRC_FP16, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q, pk, rgb, sig);
    else if (W == 128 && prec == NIRC_BF16)
        hipLaunchKernelGGL((k_infer_h16<128, NIRC_BF16, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q, pk, rgb, sig);
    else if (W == 128)
        hipLaunchKernelGGL((k_infer_h16<128, NIRC_FP16, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q, pk, rgb, sig);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_tlmc_multi_h16(int W, int prec, int mode, const BatchDesc *desc, int grid, hipStream_t s) {
    constexpr int WAVES = 8;
    static_assert(WAVES == kBatchChunkGroups, "chunk size");
    if (W != 64) return hipErrorInvalidValue;
    const bool occ = mode != NIRC_OUTPUT_RADIANCE;
    if (prec == NIRC_BF16 && !occ)
        hipLaunchKernelGGL((k_tlmc_multi_h16<64, NIRC_BF16, WAVES, false>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    else if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_tlmc_multi_h16<64, NIRC_BF16, WAVES, true>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    else if (!occ)
        hipLaunchKernelGGL((k_tlmc_multi_h16<64, NIRC_FP16, WAVES, false>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    else
        hipLaunchKernelGGL((k_tlmc_multi_h16<64, NIRC_FP16, WAVES, true>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    return hipGetLastError();
}

namespace {

struct TlmcArgs {
    Points pts;
    nirc_lobes lobes;
    const uint16_t *pk;
    int n_cache;
    DivN dn;
    uint32_t k0, k1, f;
    int mode;
    const float *rrad;
    float *tl, *c, *r;
};

template <int W, int PREC, int WAVES, bool N16>
void launch_h16_variant_n(const TlmcArgs &a, unsigned grid, hipStream_t s) {
    if (a.mode == NIRC_OUTPUT_RADIANCE)
        hipLaunchKernelGGL((k_tlmc_h16<W, PREC, WAVES, false, N16>), dim3(grid), dim3(WAVES * 64), 0, s, a.pts, a.lobes,
                           a.pk, a.n_cache, a.dn, a.k0, a.k1, a.f, a.mode, a.rrad, a.tl, a.c, a.r);
    else
        hipLaunchKernelGGL((k_tlmc_h16<W, PREC, WAVES, true, N16>), dim3(grid), dim3(WAVES * 64), 0, s, a.pts, a.lobes,
                           a.pk, a.n_cache, a.dn, a.k0, a.k1, a.f, a.mode, a.rrad, a.tl, a.c, a.r);
}

template <int W, int PREC, int WAVES>
void launch_h16_variant(const TlmcArgs &a, unsigned grid, hipStream_t s) {
    if (a.n_cache % 16 == 0) launch_h16_variant_n<W, PREC, WAVES, true>(a, grid, s);
    else launch_h16_variant_n<W, PREC, WAVES, false>(a, grid, s);
}

}  // namespace

hipError_t launch_tlmc_h16(int W, int prec, const Points &pts, const nirc_lobes &lobes, const void *packed,
                           int n_cache, uint64_t seed, uint64_t frame, int mode, const float *rrad, float *out_tl,
                           float *out_c, float *out_r, hipStream_t s) {
    constexpr int WAVES = 8;
    const unsigned grid = grid_for((pts.count + 15) / 16, WAVES, 2 * kMaxResidentBlocks);
    const TlmcArgs a{pts, lobes, (const uint16_t *)packed, n_cache, make_divn(n_cache), (uint32_t)seed,
                     (uint32_t)(seed >> 32), (uint32_t)frame, mode, rrad, out_tl, out_c, out_r};
    if (W == 64 && prec == NIRC_BF16)
        launch_h16_variant<64, NIRC_BF16, WAVES>(a, grid, s);
    else if (W == 64)
        launch_h16_variant<64, NIRC_FP16, WAVES>(a, grid, s);
    // width 128: one wave per SIMD with 4-tile passes and the hidden layers in LDS (the room of
    // four slabs beside the 96 KB of hidden-layer fragments)
    else if (W == 128 && prec == NIRC_BF16)
        launch_h16_variant<128, NIRC_BF16, 4>(a, grid_for((pts.count + 15) / 16, 4, kMaxResidentBlocks), s);
    else if (W == 128)
        launch_h16_variant<128, NIRC_FP16, 4>(a, grid_for((pts.count + 15) / 16, 4, kMaxResidentBlocks), s);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// The hash-grid model (width 64).

// packed16[e] = 16-bit(master[hash_packed_source(e)]); after an Adam step thread 0 commits it.
template <int PREC>
__global__ void k_hash_pack16(uint16_t *packed, const float *master, int64_t *step, uint32_t *flags, uint32_t *bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kHashPacked) {
        const int64_t s = hash_packed_source(e);
        packed[e] = (uint16_t)(pack2<PREC>(s >= 0 ? master[s] : 0.0f, 0.0f) & 0xFFFFu);
    }
    if (step && e == 0) {
        if (*bad) *flags |= *bad;   // the step's NIRC_FLAG_* bits
        else *step += 1;
        *bad = 0u;
    }
}

// Direction, hidden and output sections staged in LDS: [D, T0) of the hash layout.
constexpr int kHashLdsWeights = hash_sec(SEC_T0) - kHashSecD;

// Per-query inference, 16 queries per wave per iteration.
template <int PREC, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_hash_infer_h16(Points pts, Queries q, const uint16_t *__restrict__ packed,
                                                               const float2 *__restrict__ table, HashGridArgs grid,
                                                               float *__restrict__ rgb) {
    __shared__ u32x4 wsm[kHashLdsWeights / 8];
    __shared__ HashLevel s_lv[kHashLevels];
    {
        const u32x4 *src = (const u32x4 *)(packed + kHashSecD);
        for (int i = threadIdx.x; i < kHashLdsWeights / 8; i += WAVES * 64) wsm[i] = src[i];
        stage_levels(s_lv, grid);
    }
    __syncthreads();
    const uint16_t *sD = (const uint16_t *)wsm;
    const uint16_t *sH = sD + (hash_sec(SEC_H0) - kHashSecD);
    const uint16_t *sOS = sD + (hash_sec(SEC_OS) - kHashSecD);
    const uint16_t *gS = packed + kHashSecS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t Q = q.count;
    const int64_t n_tiles = (Q + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * WAVES + wave; tile < n_tiles; tile += (int64_t)gridDim.x * WAVES) {
        const int64_t qi = min((tile << 4) + col, Q - 1);
        const int64_t p = query_point(q, pts, qi);
        const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
        f32x4 h[1][4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) h[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        u32x4 b0, b1;
        float v[6], ph[15];
        hash_surface_operands<PREC>(s_lv, grid.tmask, table, xs, g, b0, b1, v, ph);
        hash_layer1_surface<PREC>(h[0], opaque(gS), b0, b1, lane);
        u32x4 bd[1][2];
        bd[0][0] = sh_operand<PREC>(q.wx[qi], q.wy[qi], q.wz[qi], g);
        bd[0][1] = u32x4{0u, 0u, 0u, 0u};
        u32x4 hb[1][2], aout[8], dfrag[8];
        load_dir_fragments<64, 1>(dfrag, sD, lane);
        mlp16<64, PREC, 1, 1>(h, hb, bd, dfrag, sH, sOS, lane, aout);
        const f32x4 z = output16_packed<64, PREC, 1>(hb, aout);
        if (col < 3) {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t qo = (tile << 4) + 4 * g + i;
                if (qo < Q) rgb[3 * qo + col] = __expf(z[i]);
            }
        }
    }
}

// Fused two-level estimator with the hash-grid model: the estimator of k_tlmc_h16 with the
// grid/phi surface part (once per point) and spherical-harmonics directions.
template <int PREC, int WAVES, bool N16>
__global__ __launch_bounds__(WAVES * 64) void k_hash_tlmc_h16(Points pts, nirc_lobes lobes,
                                                              const uint16_t *__restrict__ packed,
                                                              const float2 *__restrict__ table, HashGridArgs grid,
                                                              int n_cache, DivN dn, uint32_t key0, uint32_t key1,
                                                              uint32_t frame, const float *__restrict__ rrad,
                                                              float *__restrict__ out_tl, float *__restrict__ out_c,
                                                              float *__restrict__ out_r) {
    constexpr int SLAB = Tlmc16Lds<64>::kSlab;
    __shared__ u32x4 wsm[kHashLdsWeights / 8];
    __shared__ f32x4 slab4[WAVES * SLAB / 4];
    __shared__ nirc_lobes s_lobes;
    __shared__ HashLevel s_lv[kHashLevels];
    {
        const u32x4 *src = (const u32x4 *)(packed + kHashSecD);
        for (int i = threadIdx.x; i < kHashLdsWeights / 8; i += WAVES * 64) wsm[i] = src[i];
        if (threadIdx.x == 0) s_lobes = lobes;
        stage_levels(s_lv, grid);
    }
    __syncthreads();
    const uint16_t *sD = (const uint16_t *)wsm;
    const uint16_t *sH = sD + (hash_sec(SEC_H0) - kHashSecD);
    const uint16_t *sOS = sD + (hash_sec(SEC_OS) - kHashSecD);
    const uint16_t *gS = packed + kHashSecS;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const GroupSlab gs = group_slab((float *)slab4 + wave * SLAB, 64);
    const int64_t n_groups = (pts.count + 15) >> 4;
    const int64_t stride = (int64_t)gridDim.x * WAVES;
    // software pipeline over point groups: a group's grid corners are loaded while the previous
    // group's last queries run through the MLP (the next index is clamped to the last point, so
    // the final group's fetch stays in bounds and is simply unused)
    float2 nxt[24];
    int64_t grp = (int64_t)blockIdx.x * WAVES + __builtin_amdgcn_readfirstlane(wave);
    {
        const int64_t pc = min((grp << 4) + col, pts.count - 1);
        hash_fetch24(s_lv, grid.tmask, table, pts.px[pc], pts.py[pc], pts.pz[pc], g, nxt);
    }
    for (; grp < n_groups; grp += stride) {
        float2 cur[24];
#pragma unroll
        for (int i = 0; i < 24; ++i) cur[i] = nxt[i];
        const int64_t npc = min(((grp + stride) << 4) + col, pts.count - 1);
        tlmc_group_h16<64, PREC, 4, false, 1, false, N16>(pts, grp << 4, n_cache, dn, key0, key1, frame,
                                                          NIRC_OUTPUT_RADIANCE, rrad, out_tl, out_c, out_r, s_lobes, gS,
                                                          sD, sH, sOS, gs, lane, g, col, s_lv, grid.tmask, table, cur,
                                                          &nxt, npc);
    }
}

hipError_t launch_hash_pack16(uint16_t *packed, const float *master, int prec, hipStream_t s, int64_t *step,
                              uint32_t *flags, uint32_t *bad) {
    const dim3 grid((kHashPacked + 255) / 256), block(256);
    if (prec == NIRC_BF16)
        hipLaunchKernelGGL(k_hash_pack16<NIRC_BF16>, grid, block, 0, s, packed, master, step, flags, bad);
    else if (prec == NIRC_FP16)
        hipLaunchKernelGGL(k_hash_pack16<NIRC_FP16>, grid, block, 0, s, packed, master, step, flags, bad);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_hash_infer(int prec, const Points &pts, const Queries &q, const uint16_t *packed, const float *table,
                             const HashGridArgs &grid, float *rgb, hipStream_t s) {
    constexpr int WAVES = 4;
    const unsigned nb = grid_for((q.count + 15) / 16, WAVES, 4 * kMaxResidentBlocks);
    const float2 *t2 = (const float2 *)table;
    if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_hash_infer_h16<NIRC_BF16, WAVES>), dim3(nb), dim3(WAVES * 64), 0, s, pts, q, packed, t2,
                           grid, rgb);
    else if (prec == NIRC_FP16)
        hipLaunchKernelGGL((k_hash_infer_h16<NIRC_FP16, WAVES>), dim3(nb), dim3(WAVES * 64), 0, s, pts, q, packed, t2,
                           grid, rgb);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_hash_tlmc(int prec, const Points &pts, const nirc_lobes &lobes, const uint16_t *packed,
                            const float *table, const HashGridArgs &grid, int n_cache, uint64_t seed, uint64_t frame,
                            const float *rrad, float *out_tl, float *out_c, float *out_r, hipStream_t s) {
    constexpr int WAVES = 8;
    const unsigned nb = grid_for((pts.count + 15) / 16, WAVES, 2 * kMaxResidentBlocks);
    const float2 *t2 = (const float2 *)table;
    const DivN dn = make_divn(n_cache);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), f = (uint32_t)frame;
    const bool n16 = n_cache % 16 == 0;
    if (prec == NIRC_BF16 && n16)
        hipLaunchKernelGGL((k_hash_tlmc_h16<NIRC_BF16, WAVES, true>), dim3(nb), dim3(WAVES * 64), 0, s, pts, lobes,
                           packed, t2, grid, n_cache, dn, k0, k1, f, rrad, out_tl, out_c, out_r);
    else if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_hash_tlmc_h16<NIRC_BF16, WAVES, false>), dim3(nb), dim3(WAVES * 64), 0, s, pts, lobes,
                           packed, t2, grid, n_cache, dn, k0, k1, f, rrad, out_tl, out_c, out_r);
    else if (prec == NIRC_FP16 && n16)
        hipLaunchKernelGGL((k_hash_tlmc_h16<NIRC_FP16, WAVES, true>), dim3(nb), dim3(WAVES * 64), 0, s, pts, lobes,
                           packed, t2, grid, n_cache, dn, k0, k1, f, rrad, out_tl, out_c, out_r);
    else if (prec == NIRC_FP16)
        hipLaunchKernelGGL((k_hash_tlmc_h16<NIRC_FP16, WAVES, false>), dim3(nb), dim3(WAVES * 64), 0, s, pts, lobes,
                           packed, t2, grid, n_cache, dn, k0, k1, f, rrad, out_tl, out_c, out_r);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace nirc
