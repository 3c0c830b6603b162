// Shared device routines of the MLP layer chain (FP32 MFMA 16x16x4) and the launcher interface
// used by the C ABI.
#pragma once

#include "nirc_device.hpp"

namespace nirc {

// Upper bound of resident workgroups used for grid-stride launches (256 CUs).
constexpr int kMaxResidentBlocks = 256;

// Width-64 weights are staged in LDS once per workgroup; width 128 would not leave room for
// the per-wave slabs (the FP32 hidden layers alone are 192 KB), so those kernels read their
// weight fragments from global memory (L2-resident) inside each pass.
__host__ __device__ constexpr bool lds_weights(int W) { return W <= 64; }

template <int W>
struct InferLds {
    // first-layer direction columns, three hidden layers and the output layer, in packed order
    static constexpr int kWeights = F32Layout{W}.offset(SEC_T0) - F32Layout{W}.offset(SEC_D);
};

// Staged directions per wave: 8 tiles of 16, plus one more tile when a point group's residual
// tile is generated together with its last 8 cache tiles (N a multiple of 8).
constexpr int kDirSlots = 144;

template <int W>
struct TlmcLds {
    // h_s of 16 points, 128 staged directions, per-point cache sums [16][4], residual
    // predictions [16][4] and a per-tile query buffer [16][4] (the FP32 estimator keeps its sums
    // in registers and puts the group's normals [3][16] there instead)
    static constexpr int kSlab = 16 * W + 3 * kDirSlots + 3 * 64;
};

// Orders this wave's LDS traffic for an exchange between its own lanes without waiting for
// outstanding LDS loads: a wave's LDS instructions execute in issue order, so only the compiler
// has to be kept from moving the accesses across this point.
__device__ inline void wave_lds_order() {
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// Orders this wave's LDS traffic around a point where lanes exchange data through LDS.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Returns p unchanged but opaque to the optimiser, so that weight loads inside a loop are not
// hoisted out of it (hoisting every fragment load would need hundreds of registers).
// Only for pointers to global memory: the result is rebuilt in the global address space, so
// loads through it stay global loads.
template <typename T>
__device__ __forceinline__ const T *opaque(const T *p) {
    uint64_t v = (uint64_t)p;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    typedef const T __attribute__((address_space(1))) *global_ptr;
    return (const T *)(global_ptr)(((uint64_t)hi << 32) | lo);
}

// A pointer that holds the same value in every lane, moved to scalar registers so that a branch
// on it is taken by the whole wave (no divergent join).
__device__ __forceinline__ const float *uniform_ptr(const float *p) {
    const uint64_t v = (uint64_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (const float *)(((uint64_t)hi << 32) | lo);
}

// h += W1_s e_s for one 16-column tile; the surface features are computed here in B layout.
template <int W>
__device__ __forceinline__ void layer1_surface(f32x4 (&h)[W / 16], const float *gS, const float xs[7],
                                               int lane, int g) {
    constexpr int MT = W / 16;
#pragma unroll
    for (int kq = 0; kq < 7; ++kq) {
        float b[4];
        enc_pair2(xs[kq], 2 * g, b[0], b[1], b[2], b[3]);
        f32x4 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(gS + ((mt * 7 + kq) * 64 + lane) * 4);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) h[mt] = mfma4(a[mt][kk], b[kk], h[mt]);
    }
}

// h[tt] += W1_w e_w(direction of tile tt) for up to T tiles (nt valid).
template <int W, int T>
__device__ __forceinline__ void layer1_direction(f32x4 (&h)[T][W / 16], const float *sD, const float *dx,
                                                 const float *dy, const float *dz, int lane, int g) {
    constexpr int MT = W / 16;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        float b[T][4];
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const float v = i == 0 ? dx[tt] : i == 1 ? dy[tt] : dz[tt];
            enc_pair2(v, 2 * g, b[tt][0], b[tt][1], b[tt][2], b[tt][3]);
        }
        f32x4 a[MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sD + ((mt * 3 + i) * 64 + lane) * 4);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma4(a[mt][kk], b[tt][kk], h[tt][mt]);
    }
}

template <int W, int T>
__device__ __forceinline__ void relu_all(f32x4 (&h)[T][W / 16]) {
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int mt = 0; mt < W / 16; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i) h[tt][mt][i] = relu_f32(h[tt][mt][i]);
}

// Hidden layers 2..4: K-quad kq of the packed fragments is exactly row tile kq of the previous
// layer's result, so register (tt, kq, kk) feeds K-block 4 kq + kk.
template <int W, int T>
__device__ __forceinline__ void hidden_layers(f32x4 (&h)[T][W / 16], const float *sH, int lane) {
    constexpr int MT = W / 16, KQ = W / 16;
    constexpr int SEC = MT * (W / 4) * 64;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        // keep each layer's fragment loads inside the layer (hoisting them all costs registers)
        __builtin_amdgcn_sched_barrier(0);
        const float *sec = sH + l * SEC;
        f32x4 o[T][MT];
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) o[tt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        // the layer's MFMA run at raised issue priority (the SIMD's other wave fills the gaps)
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int kq = 0; kq < KQ; ++kq) {
            f32x4 a[MT];
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int tt = 0; tt < T; ++tt) o[tt][mt] = mfma4(a[mt][kk], h[tt][kq][kk], o[tt][mt]);
        }
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) h[tt][mt][i] = relu_f32(o[tt][mt][i]);
    }
}

// Output layer (rows 0..2 of a 16-row tile): lanes 0..15 receive z = W5 h4 of their column.
template <int W, int T>
__device__ __forceinline__ void output_layer(f32x4 (&y)[T], const f32x4 (&h)[T][W / 16], const float *sO,
                                             int lane) {
    constexpr int KQ = W / 16;
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int tt = 0; tt < T; ++tt) y[tt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kq = 0; kq < KQ; ++kq) {
        const f32x4 a = *(const f32x4 *)(sO + (kq * 64 + lane) * 4);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int tt = 0; tt < T; ++tt) y[tt] = mfma4(a[kk], h[tt][kq][kk], y[tt]);
    }
}

// ------------------------------------------------------------------------------------------
// Pieces of the fused estimator shared by all precisions.

// Cosine-weighted direction from uniforms (u1, u2) about a unit normal, with the hardware sine
// and cosine of 2 pi u2 (argument in revolutions; absolute error ~1e-6, far below the 16-bit
// operands the direction feeds).  Used for the cache directions of the 16-bit estimators, whose
// directions never leave the kernel; residual directions keep the exact map of cosine_dir.
__device__ __forceinline__ void cosine_dir_fast(float nx, float ny, float nz, float u1, float u2, float &wx,
                                                float &wy, float &wz) {
#pragma clang fp contract(off)
    const float r = __builtin_amdgcn_sqrtf(u1);
    const float lx = r * __builtin_amdgcn_cosf(u2), ly = r * __builtin_amdgcn_sinf(u2);
    const float lz = __builtin_amdgcn_sqrtf(1.0f - u1);
    const float s = nz >= 0.0f ? 1.0f : -1.0f;
    const float a = -__builtin_amdgcn_rcpf(s + nz);
    const float b = nx * ny * a;
    const float tx = 1.0f + s * nx * nx * a, ty = s * b, tz = -s * nx;
    const float by = s + ny * ny * a;
    wx = lx * tx + ly * b + lz * nx;
    wy = lx * ty + ly * by + lz * ny;
    wz = lx * tz - ly * ny + lz * nz;
}

// The estimators' direction batch: the directions of tiles tb .. tb + 7 of a point group (with
// `fold`, also the residual tile after them) into the slab's slots db [3][kDirSlots], one Philox
// block per lane giving two directions (the counters of dir_counter), with the group's normals
// read from the slab (nrm [3][16], staged once per group) and 32-bit point indices (point counts
// stay below 2^31).  FAST (the 16-bit estimators):
// cache directions by the fast map; residual directions (tile n_cache, and the folded residual
// tile) always use the exact map, so that they equal the directions tlmc_sample_dirs returns.
template <bool FAST>
__device__ __forceinline__ void gen_dirs_batch_nrm(uint32_t p0, int tb, int n_cache, DivN dn, uint32_t key0,
                                                 uint32_t key1, uint32_t frame, int lane, float *db, const float *nrm,
                                                 bool fold) {
    const int T = tb + (lane >> 3);
    const int c0 = (2 * lane) & 15;
    float wa[3] = {0.f, 0.f, 0.f}, wb[3] = {0.f, 0.f, 0.f};
    if (T <= n_cache) {
        const bool res = (T == n_cache);
        int ja, jb, ka = 0, kb = 0;
        if (res) {
            ja = c0;
            jb = c0 + 1;
        } else {
            const int qa = 16 * T + c0;
            ja = (int)div_n((uint32_t)qa, dn);
            ka = qa - ja * n_cache;
            jb = (int)div_n((uint32_t)(qa + 1), dn);
            kb = qa + 1 - jb * n_cache;
        }
        const DirCounter ca = dir_counter(p0 + (uint32_t)ja, ka, res);
        const DirCounter cb = dir_counter(p0 + (uint32_t)jb, kb, res);
        const Rand4 ra = philox(ca.c0, ca.c1, frame, ca.stream, key0, key1);
        Rand4 rb = ra;
        if (ca.c0 != cb.c0 || ca.c1 != cb.c1)   // only for odd N
            rb = philox(cb.c0, cb.c1, frame, cb.stream, key0, key1);
        const float nax = nrm[ja], nay = nrm[16 + ja], naz = nrm[32 + ja];
        const float nbx = nrm[jb], nby = nrm[16 + jb], nbz = nrm[32 + jb];
        const float ua1 = u24(ca.half ? ra.r[2] : ra.r[0]), ua2 = u24(ca.half ? ra.r[3] : ra.r[1]);
        const float ub1 = u24(cb.half ? rb.r[2] : rb.r[0]), ub2 = u24(cb.half ? rb.r[3] : rb.r[1]);
        if (!FAST || res) {
            cosine_dir(nax, nay, naz, ua1, ua2, wa[0], wa[1], wa[2]);
            cosine_dir(nbx, nby, nbz, ub1, ub2, wb[0], wb[1], wb[2]);
        } else {
            cosine_dir_fast(nax, nay, naz, ua1, ua2, wa[0], wa[1], wa[2]);
            cosine_dir_fast(nbx, nby, nbz, ub1, ub2, wb[0], wb[1], wb[2]);
        }
    }
    // residual direction of point rl = lane % 16 of the group (exact map): every lane computes
    // that of its rl and all lanes store the same value
    float ra_[3] = {0.f, 0.f, 0.f};
    const int rl = lane & 15;
    if (fold) {
        const DirCounter c = dir_counter(p0 + (uint32_t)rl, 0, true);
        const Rand4 r = philox(c.c0, c.c1, frame, c.stream, key0, key1);
        dir_from_rand(r, c.half, nrm[rl], nrm[16 + rl], nrm[32 + rl], ra_[0], ra_[1], ra_[2]);
    }
    wave_sync();   // the previous batch's readers are done
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        db[kDirSlots * d + 2 * lane] = wa[d];
        db[kDirSlots * d + 2 * lane + 1] = wb[d];
    }
    if (fold) {
#pragma unroll
        for (int d = 0; d < 3; ++d) db[kDirSlots * d + 128 + rl] = ra_[d];
    }
    wave_sync();
}

// Sums over aligned groups of 2, 4, 8 or 16 lanes of a 16-lane row with DPP (result in every
// lane of the group): quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror.
__device__ __forceinline__ float dpp_add(float x, int ctrl_step) {
    const int v = __builtin_bit_cast(int, x);
    int r;
    switch (ctrl_step) {
    case 0: r = __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true); break;
    case 1: r = __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true); break;
    case 2: r = __builtin_amdgcn_mov_dpp(v, 0x141, 0xF, 0xF, true); break;
    default: r = __builtin_amdgcn_mov_dpp(v, 0x140, 0xF, 0xF, true); break;
    }
    return x + __builtin_bit_cast(float, r);
}

// Cache tile T: lanes 0..15 hold y of queries 16 T + column; point `col` (lanes 0..15) adds the
// sum of its queries in this tile.  N a multiple of 16: the tile belongs to one point and a DPP
// row sum suffices; N dividing 16: DPP segment sums and one cross-lane read; any other N:
// 16-lane inclusive prefix sums.
// N16: n_cache is known to be a multiple of 16 (only the first path is compiled).
template <bool N16 = false>
__device__ __forceinline__ void reduce_cache_tile(int T, int n_cache, int col, float y0, float y1, float y2,
                                                  float &fc0, float &fc1, float &fc2) {
    if (N16 || (n_cache & 15) == 0) {
#pragma unroll
        for (int st = 0; st < 4; ++st) {
            y0 = dpp_add(y0, st);
            y1 = dpp_add(y1, st);
            y2 = dpp_add(y2, st);
        }
        if (col == (16 * T) / n_cache) {
            fc0 += y0;
            fc1 += y1;
            fc2 += y2;
        }
        return;
    }
    if constexpr (!N16) {
        if (n_cache < 16 && (16 % n_cache) == 0) {
            const int steps = n_cache == 8 ? 3 : n_cache == 4 ? 2 : n_cache == 2 ? 1 : 0;
            for (int st = 0; st < steps; ++st) {
                y0 = dpp_add(y0, st);
                y1 = dpp_add(y1, st);
                y2 = dpp_add(y2, st);
            }
            // point `col` is segment (col - 16T/N) of this tile if that lies in [0, 16/N)
            const int seg = col - (16 * T) / n_cache;
            const bool mine = seg >= 0 && seg < 16 / n_cache;
            const int src = mine ? seg * n_cache : 0;
            const float s0 = __shfl(y0, src, 16), s1 = __shfl(y1, src, 16), s2 = __shfl(y2, src, 16);
            if (mine) {
                fc0 += s0;
                fc1 += s1;
                fc2 += s2;
            }
            return;
        }
        float s0 = y0, s1 = y1, s2 = y2;
#pragma unroll
        for (int d = 1; d < 16; d <<= 1) {
            const float u0 = __shfl_up(s0, d, 16);
            const float u1 = __shfl_up(s1, d, 16);
            const float u2 = __shfl_up(s2, d, 16);
            if (col >= d) {
                s0 += u0;
                s1 += u1;
                s2 += u2;
            }
        }
        // point `col` owns queries [col N, col N + N) -> columns [lo, hi)
        const int a = col * n_cache - 16 * T;
        const int lo = max(a, 0), hi = min(a + n_cache, 16);
        const int shi = min(max(hi - 1, 0), 15), slo = min(max(lo - 1, 0), 15);
        const float h0 = __shfl(s0, shi, 16), l0 = __shfl(s0, slo, 16);
        const float h1 = __shfl(s1, shi, 16), l1 = __shfl(s1, slo, 16);
        const float h2 = __shfl(s2, shi, 16), l2 = __shfl(s2, slo, 16);
        if (lo < hi) {
            fc0 += lo > 0 ? h0 - l0 : h0;
            fc1 += lo > 0 ? h1 - l1 : h1;
            fc2 += lo > 0 ? h2 - l2 : h2;
        }
    }
}

__device__ __forceinline__ void store_estimate(int64_t p, float inv_n, float fc0, float fc1, float fc2, float fr0,
                                               float fr1, float fr2, float *out_tl, float *out_c, float *out_r) {
    const int64_t o = 3 * p;
    const float c0 = fc0 * inv_n, c1 = fc1 * inv_n, c2 = fc2 * inv_n;
    out_tl[o + 0] = c0 + fr0;
    out_tl[o + 1] = c1 + fr1;
    out_tl[o + 2] = c2 + fr2;
    if (out_c) {
        out_c[o + 0] = c0;
        out_c[o + 1] = c1;
        out_c[o + 2] = c2;
    }
    if (out_r) {
        out_r[o + 0] = fr0;
        out_r[o + 1] = fr1;
        out_r[o + 2] = fr2;
    }
}

// ------------------------------------------------------------------------------------------
// Work list of the batched estimator (device memory; written by the host).
constexpr int kBatchChunkGroups = 8;   // point groups (of 16 points) per chunk = waves per workgroup
constexpr int kBatchMaxRequests = 64;

struct BatchRequest {
    Points pts;
    const void *packed;   // the request's packed weights (precision of the batch)
    nirc_lobes lobes;
    int32_t n_cache;
    DivN dn;
    uint32_t key0, key1, frame;
    const float *rrad;     // residual radiance [P][3], or NULL for the field
    int32_t mode;          // NIRC_OUTPUT_* of the model
    float *out_tl, *out_c, *out_r;
    int32_t chunk_begin;   // first chunk of this request in the batch
    int32_t pad;
};

struct BatchDesc {
    int32_t n_requests;
    int32_t total_chunks;
    int32_t width;
    int32_t precision;
    BatchRequest req[kBatchMaxRequests];
};

// Work list of a batched training step (several models, each with its own samples, workspace
// and state): built on the host, read by the multi-request training kernels.
struct TrainReq {
    Points pts;
    nirc_lobes lobes;
    const uint16_t *packed16;            // the model's 16-bit copy (rewritten by the step)
    float *master, *m, *v;
    int64_t *step;
    uint32_t *flags, *bad;
    float *partials, *lpart, *grad, *loss;   // the model's workspace (WorkLayout of its batch)
    int32_t *sp;                         // samples: point [B], wx, wy, wz [B], target [B][3]
    float *swx, *swy, *swz, *stgt;
    int64_t batch;
    uint32_t key0, key1, frame;
    int32_t nb;                          // gradient blocks of this request
    int32_t vb0;                         // its first virtual block in the list
    float lr, b1, b2, eps, loss_eps, loss_scale;
    int32_t loss_kind, output;
    float *dyn_scale;                    // FP16: the model's dynamic loss scale, else NULL
    uint32_t *good_steps;                // FP16: finite steps since the last change of the scale
    uint32_t *done;                      // the model's count of finished Adam workgroups (zero between steps)
};

struct TrainDesc {
    int32_t n;
    int32_t total_vb;
    int32_t width;
    int32_t precision;
    int64_t max_batch;
    int64_t pad;
    TrainReq req[kBatchMaxRequests];
};

// ------------------------------------------------------------------------------------------
// Launchers (return the launch status).
hipError_t launch_pack(float *packed, const float *master, int W, hipStream_t s);
// Packs the 16-bit copy; with step/flags/bad (after Adam) it also commits the step.
hipError_t launch_pack16(uint16_t *packed, const float *master, int W, int prec, hipStream_t s,
                         int64_t *step = nullptr, uint32_t *flags = nullptr, uint32_t *bad = nullptr,
                         float *dyn_scale = nullptr, uint32_t *good_steps = nullptr);
hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s);
hipError_t launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s);
hipError_t launch_encode(const Points &pts, const Queries &q, float *feat, hipStream_t s);
hipError_t launch_sample_dirs(const Points &pts, int n_cache, uint64_t seed, uint64_t frame,
                              float *dirs, hipStream_t s);
// Training samples of steps step .. step + nsteps - 1 in one launch; step k's buffers start
// (k - step) * stride elements after the given ones.
hipError_t launch_train_batch(const Points &pts, const nirc_lobes &lobes, int64_t batch,
                              uint64_t seed, uint64_t frame, uint32_t step, int mode, int32_t *point,
                              float *wx, float *wy, float *wz, float *target, hipStream_t s, int nsteps = 1,
                              int64_t stride = 0);
// Steps of a training frame whose samples one launch makes (the workspace holds them).
constexpr int kFrameSampleSteps = 4;
// Reference integral of V L over the hemisphere (tensor Gauss-Legendre on the cosine map's
// uniforms; nodes and weights on [0, 1] from the host), FP64 [P][3].
constexpr int kMaxQuadNodes = 128;
struct QuadNodes {
    double x[kMaxQuadNodes], w[kMaxQuadNodes];
    int n;
};
hipError_t launch_reference_occluded(const Points &pts, const nirc_lobes &lobes, const QuadNodes &nodes, double *F,
                                     hipStream_t s);
unsigned grid_for(int64_t units, int waves, int max_blocks);
// mode: the output mode shared by every request of the list (NIRC_OUTPUT_*)
hipError_t launch_tlmc_multi_h16(int W, int prec, int mode, const BatchDesc *desc, int grid, hipStream_t s);
hipError_t launch_tlmc_multi_f32(int W, int mode, const BatchDesc *desc, int grid, hipStream_t s);
hipError_t launch_infer_h16(int W, int prec, const Points &pts, const Queries &q, const void *packed, float *rgb,
                            int sig, hipStream_t s);
hipError_t launch_tlmc_h16(int W, int prec, const Points &pts, const nirc_lobes &lobes, const void *packed,
                           int n_cache, uint64_t seed, uint64_t frame, int mode, const float *rrad, float *out_tl,
                           float *out_c, float *out_r, hipStream_t s);
// sig: sigmoid outputs (the visibility cache) instead of exp
hipError_t launch_infer(int W, int prec, const Points &pts, const Queries &q, const void *packed, float *rgb,
                        int sig, hipStream_t s);
// Biased estimate (balanced termination heuristic) from F_c written by launch_tlmc: out [P][3],
// cont [P] (1 = the path continues) or NULL.
hipError_t launch_bth(const Points &pts, const nirc_lobes &lobes, int n_cache, uint64_t seed, uint64_t frame,
                      int mode, const float *rrad, const float *fc, float *out, int32_t *cont, hipStream_t s);
// rrad: residual radiance [P][3] (a renderer's sample), or NULL to evaluate the lobe field
// mode: NIRC_OUTPUT_* (the visibility cache multiplies its predictions by the field; the occluded
// modes take V L as the residual sample)
hipError_t launch_tlmc(int W, int prec, const Points &pts, const nirc_lobes &lobes, const void *packed,
                       int n_cache, uint64_t seed, uint64_t frame, int mode, const float *rrad, float *out_tl,
                       float *out_c, float *out_r, hipStream_t s);

// Frame statistics (FP64).
hipError_t launch_reference_table(const nirc_lobes &lobes, double *table, hipStream_t s);
hipError_t launch_reference(const Points &pts, const nirc_lobes &lobes, const double *table, double *F,
                            hipStream_t s);
hipError_t launch_frame_stats(const Points &pts, const nirc_lobes &lobes, const double *table, const float *tl,
                              const float *fc, const float *fr, double eps, double *scratch, double *stats,
                              hipStream_t s);
size_t frame_stats_scratch_bytes();
hipError_t launch_accumulate(const float *v, int64_t n, double *sum, double *sumsq, hipStream_t s);

// Training (gradient partials, reduction, Adam).
struct TrainArgs {
    const float *target;   // [B][3] for the loss, or NULL
    const float *d_rgb;    // [B][3] upstream gradient for the VJP, or NULL
    float loss_eps;
    float loss_scale;
    int32_t loss_kind;     // NIRC_LOSS_*
    const float *fr;       // NIRC_LOSS_VAR: batch estimate of F_r per channel [3], else NULL
    int32_t sig;           // sigmoid outputs (the visibility cache) instead of exp
    const float *dyn_scale;   // FP16 models: the current dynamic loss scale (device), which
                              // replaces loss_scale as dyn_scale * B; NULL: loss_scale as given
};

// Dynamic loss scaling of FP16 models: a step skipped for a non-finite gradient halves the scale,
// kLossScaleGrowth finite steps in a row double it, within [kLossScaleMin, kLossScaleMax].
constexpr uint32_t kLossScaleGrowth = 1000;
constexpr float kLossScaleMin = 0x1p-14f, kLossScaleMax = 0x1p24f;

// Threads per workgroup of the one-launch Adam kernels (one parameter per thread): fewer
// workgroups count themselves into the finished-workgroup counter one after another (a 4-step
// width-64 training frame measured 0.246 / 0.231 / 0.222 / 0.216 / 0.216 ms with 64 / 128 / 256 /
// 512 / 1024 threads in BF16).
constexpr int kAdamThreads = 512;

// Adam (Kingma & Ba) for one parameter with bias correction at t = step + 1 (c1 = 1 - b1^t,
// c2 = 1 - b2^t): updates the moments m and v from gradient g and returns the new weight.  Every
// Adam kernel uses this one expression with every product and sum rounded on its own (no fused
// multiply-adds, which the compiler could otherwise form differently in different kernels), so
// that all of them produce the same bits.
__device__ __forceinline__ float adam_update(float w, float &m, float &v, float g, float c1, float c2, float lr,
                                             float b1, float b2, float eps) {
#pragma clang fp contract(off)
    m = b1 * m + (1.0f - b1) * g;
    v = b2 * v + (1.0f - b2) * g * g;
    return w - lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// The commit of a training step, by the one thread that finishes it: a step flagged in `bad`
// records its NIRC_FLAG_* bits in `flags` and, for a non-finite gradient with a dynamic loss
// scale, halves the scale; a finite step advances the step count and, after kLossScaleGrowth
// of them in a row, doubles the scale.  Clears `bad` for the next step.
__device__ inline void commit_step(int64_t *step, uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good) {
    const uint32_t b = *bad;
    if (b) {
        *flags |= b;
        if (dyn_scale && (b & NIRC_FLAG_NONFINITE_GRAD)) {   // back off
            *dyn_scale = fmaxf(*dyn_scale * 0.5f, kLossScaleMin);
            *good = 0u;
        }
    } else {
        *step += 1;
        if (dyn_scale && ++*good >= kLossScaleGrowth) {
            *dyn_scale = fminf(*dyn_scale * 2.0f, kLossScaleMax);
            *good = 0u;
        }
    }
    *bad = 0u;
}

// NIRC_LOSS_VAR: fr[c] = mean over the batch of t - y (y: the model's predictions [B][3]),
// summed in a fixed order; part holds kFrBlocks x 3 floats.
constexpr int kFrBlocks = 256;
hipError_t launch_residual_mean(const float *y, const float *t, int64_t B, float *part, float *fr, hipStream_t s);
int train_blocks(int64_t batch);     // workgroups used by the FP32 gradient kernel for a batch
int train_blocks16(int64_t batch);   // workgroups used by the 16-bit gradient kernel
hipError_t launch_grad_partials16(int W, int prec, const Points &pts, const Queries &q, const void *packed,
                                  TrainArgs a, float *partials, float *loss_partials, int nblocks, hipStream_t s);
hipError_t launch_grad_partials(int W, const Points &pts, const Queries &q, const float *packed,
                                TrainArgs a, float *partials, float *loss_partials, int nblocks,
                                hipStream_t s);
// dyn_scale (nullable): the gradient is divided by dyn_scale * dyn_batch instead of multiplied by
// inv_scale.
hipError_t launch_reduce_grad(int W, const float *partials, const float *loss_partials, int nblocks,
                              float inv_scale, float loss_norm, float *grad, float *loss,
                              uint32_t *bad, hipStream_t s, const float *dyn_scale = nullptr, float dyn_batch = 1.0f);
hipError_t launch_check_finite(int W, const float *grad, uint32_t *bad, hipStream_t s);
hipError_t launch_reduce_grad_n(int64_t np, const float *partials, const float *loss_partials, int nblocks,
                                float inv_scale, float loss_norm, float *grad, float *loss, uint32_t *bad,
                                hipStream_t s);
hipError_t launch_check_finite_n(int64_t np, const float *grad, uint32_t *bad, hipStream_t s);
hipError_t launch_adam_n(int64_t np, float *master, float *m, float *v, const float *grad, const int64_t *step,
                         const uint32_t *bad, float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_scale_check(float *g, int64_t n, float scale, uint32_t *bad, hipStream_t s);
// Adam on the master weights, the refresh of the copy the kernels read (the FP32 copy for FP32
// models, only the 16-bit copy for 16-bit models) and the step commit, in one launch (`done` its
// workgroup counter, zero between steps).
hipError_t launch_adam(int W, float *master, float *m, float *v, const float *grad, int64_t *step,
                       uint32_t *flags, uint32_t *bad, float lr, float b1, float b2, float eps,
                       float *packed, uint16_t *packed16, int prec, hipStream_t s, uint32_t *done,
                       float *dyn_scale = nullptr, uint32_t *good_steps = nullptr);
// One training step of every request of a device work list (width 64, 16-bit models): samples
// of step `step`, gradient partials, reduction, Adam and the 16-bit repack with the step commit.
// Launch shapes depend only on the list's capacity, so the sequence can be captured in a graph
// and replayed over other lists.
hipError_t launch_train_step_multi(const TrainDesc *desc, int prec, uint32_t step, int64_t max_batch, hipStream_t s);
hipError_t launch_train_batch_multi(const TrainDesc *desc, uint32_t step, int64_t max_batch, hipStream_t s);
// The estimator with its fusions undone (stages 0..2; 16-bit, width 64), for measuring them.
size_t ablation_workspace_bytes(int64_t P, int n_cache, int stage);
hipError_t launch_ablation(int prec, int stage, const Points &pts, const nirc_lobes &lobes, const uint16_t *packed,
                           int n_cache, uint64_t seed, uint64_t frame, char *ws, float *out_tl, float *out_c,
                           float *out_r, hipStream_t s);
hipError_t launch_reduce_grad_multi(const TrainDesc *desc, int W, hipStream_t s);
// Adam with the 16-bit copy refreshed in the same pass and the step committed by the last
// workgroup (done: a counter that is zero between steps).
hipError_t launch_adam_pack16(int W, int prec, float *w, float *m, float *v, const float *grad, int64_t *step,
                              uint32_t *flags, uint32_t *bad, float *dyn_scale, uint32_t *good, uint32_t *done,
                              uint16_t *packed, float lr, float b1, float b2, float eps, hipStream_t s);
hipError_t launch_adam_pack16_multi(const TrainDesc *desc, int W, int prec, hipStream_t s);

}  // namespace nirc
