// Inference-side kernels: weight packing, input encoding, direction sampling, training-sample
// generation, per-query cache inference and the fused two-level estimator.
#include "nirc_hash.hpp"

namespace nirc {

// ------------------------------------------------------------------------------------------
// Small utilities

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy_f32(float *dst, const float *src, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// packed[e] = master[source(e)] (zero padding where the fragment has no weight).
__global__ void k_pack_f32(float *packed, const float *master, int W, int total) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= total) return;
    const int64_t s = f32_packed_source(W, e);
    packed[e] = s >= 0 ? master[s] : 0.0f;
}

// ------------------------------------------------------------------------------------------
// Encoding: one thread per (query, input); 16 features each, canonical order.
__global__ void k_encode(Points pts, Queries q, float *feat) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= q.count * kInputs) return;
    const int64_t qi = t / kInputs;
    const int i = (int)(t - qi * kInputs);
    const int64_t p = query_point(q, pts, qi);
    float v;
    switch (i) {
    case 0: v = pts.px[p]; break;
    case 1: v = pts.py[p]; break;
    case 2: v = pts.pz[p]; break;
    case 3: v = q.wx[qi]; break;
    case 4: v = q.wy[qi]; break;
    case 5: v = q.wz[qi]; break;
    case 6: v = pts.nx[p]; break;
    case 7: v = pts.ny[p]; break;
    case 8: v = pts.nz[p]; break;
    default: v = pts.rough[p]; break;
    }
    float *o = feat + qi * kFeat + 16 * i;
    if (!point_index_ok(q, pts, qi)) {   // no point to encode: the query's features are NaN
#pragma unroll
        for (int k = 0; k < 2 * kFreq; ++k) o[k] = __builtin_nanf("");
        return;
    }
#pragma unroll
    for (int k = 0; k < kFreq; ++k) enc_pair(v, k, o[2 * k], o[2 * k + 1]);
}

// ------------------------------------------------------------------------------------------
// Sampled directions, one thread per (point, k): [P][N+1][3], entry N = residual.
__global__ void k_sample_dirs(Points pts, int n_cache, uint32_t key0, uint32_t key1,
                              uint32_t frame, float *dirs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t per = n_cache + 1;
    if (t >= pts.count * per) return;
    const int64_t p = t / per;
    const int k = (int)(t - p * per);
    const DirCounter c = dir_counter((uint32_t)p, k, k == n_cache);
    const Rand4 r = philox(c.c0, c.c1, frame, c.stream, key0, key1);
    float wx, wy, wz;
    dir_from_rand(r, c.half, pts.nx[p], pts.ny[p], pts.nz[p], wx, wy, wz);
    dirs[3 * t + 0] = wx;
    dirs[3 * t + 1] = wy;
    dirs[3 * t + 2] = wz;
}

// Biased estimate with the balanced termination heuristic at the shading point, one thread per
// point, after the fused estimator has written F_c: the path's scattering direction is the
// residual direction (same Philox stream, same FP32 map, so the same direction as the fused
// kernel's), P_s = cos / (cos + N) for the cosine pdf, and xi (counter (p >> 2, 0, frame, 6),
// word p & 3) stops the path when xi > P_s, i.e. when (xi N)^2 > (1 - u1) (1 - xi)^2 with
// cos = sqrt(1 - u1): FP64 products of exact 24-bit uniforms, so the decision does not depend
// on the FP32 rounding of the direction.  Stopped: F_c; continued: the radiance along the
// direction (rrad, or the field).
__global__ void k_bth(Points pts, nirc_lobes lobes, int n_cache, uint32_t key0, uint32_t key1, uint32_t frame,
                      int mode, const float *__restrict__ rrad, const float *__restrict__ fc,
                      float *__restrict__ out, int32_t *__restrict__ cont) {
#pragma clang fp contract(off)
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= pts.count) return;
    const DirCounter dc = dir_counter((uint32_t)p, n_cache, true);
    const Rand4 r = philox(dc.c0, dc.c1, frame, dc.stream, key0, key1);
    const Rand4 rt = philox((uint32_t)p >> 2, 0u, frame, (uint32_t)kStreamTerminate, key0, key1);
    const int q = (int)(p & 3);
    const uint32_t word = q == 0 ? rt.r[0] : q == 1 ? rt.r[1] : q == 2 ? rt.r[2] : rt.r[3];
    // xi > cos / (cos + N) with cos = sqrt(1 - u1), xi = X 2^-24, u1 = U 2^-24 (24-bit integers):
    // (X N)^2 2^24 > (2^24 - U) (2^24 - X)^2, both sides exact in 128-bit integers (X N < 2^36).
    const uint64_t X = word >> 8, U = (dc.half ? r.r[2] : r.r[0]) >> 8;
    const uint64_t xn = X * (uint64_t)n_cache, xc = (1ull << 24) - X;
    const bool stop = ((unsigned __int128)xn * xn << 24) > (unsigned __int128)((1ull << 24) - U) * (xc * xc);
    if (cont) cont[p] = stop ? 0 : 1;
    float v[3];
    if (stop) {
        v[0] = fc[3 * p];
        v[1] = fc[3 * p + 1];
        v[2] = fc[3 * p + 2];
    } else if (rrad) {
        v[0] = rrad[3 * p];
        v[1] = rrad[3 * p + 1];
        v[2] = rrad[3 * p + 2];
    } else {
        float wx, wy, wz;
        dir_from_rand(r, dc.half, pts.nx[p], pts.ny[p], pts.nz[p], wx, wy, wz);
        field_eval(lobes, pts.px[p], pts.py[p], pts.pz[p], wx, wy, wz, v);
        if (mode != NIRC_OUTPUT_RADIANCE) {   // the continued path meets the occluder
            const float V = visibility(lobes, pts.px[p], wx, wy, wz);
            v[0] *= V;
            v[1] *= V;
            v[2] *= V;
        }
    }
    out[3 * p] = v[0];
    out[3 * p + 1] = v[1];
    out[3 * p + 2] = v[2];
}

// Reference integral of the occluded scene, one workgroup per point: the n x n tensor
// Gauss-Legendre nodes over the cosine map's uniforms (u1, u2), FP32 integrand V L, FP64 sums in a
// fixed order (strided per thread, then a tree).
__global__ __launch_bounds__(256) void k_reference_occluded(Points pts, nirc_lobes lobes, QuadNodes nodes,
                                                            double *__restrict__ F) {
    __shared__ double sh[3][256];
    const int64_t p = blockIdx.x;
    const float x0 = pts.px[p], x1 = pts.py[p], x2 = pts.pz[p];
    const float nx = pts.nx[p], ny = pts.ny[p], nz = pts.nz[p];
    const int n = nodes.n, nn = n * n;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    for (int t = threadIdx.x; t < nn; t += 256) {
        const int i = t / n, k = t - i * n;
        float wx, wy, wz, L[3];
        cosine_dir(nx, ny, nz, (float)nodes.x[i], (float)nodes.x[k], wx, wy, wz);
        field_eval(lobes, x0, x1, x2, wx, wy, wz, L);
        const double wt = nodes.w[i] * nodes.w[k] * (double)visibility(lobes, x0, wx, wy, wz);
        a0 += wt * (double)L[0];
        a1 += wt * (double)L[1];
        a2 += wt * (double)L[2];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) F[3 * p + threadIdx.x] = sh[threadIdx.x][0];
}

hipError_t launch_reference_occluded(const Points &pts, const nirc_lobes &lobes, const QuadNodes &nodes, double *F,
                                     hipStream_t s) {
    if (pts.count == 0) return hipSuccess;
    if (nodes.n < 1 || nodes.n > kMaxQuadNodes || pts.count > INT32_MAX) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reference_occluded, dim3((unsigned)pts.count), dim3(256), 0, s, pts, lobes, nodes, F);
    return hipGetLastError();
}

// Training samples: one thread per sample.
__device__ __forceinline__ void train_sample(const Points &pts, const nirc_lobes &lobes, uint32_t key0, uint32_t key1,
                                             uint32_t frame, uint32_t step, int mode, int64_t b, int32_t *point,
                                             float *wx, float *wy, float *wz, float *target) {
    const Rand4 r = philox((uint32_t)b, step, frame, (uint32_t)kStreamTrain, key0, key1);
    const int64_t p = (int64_t)(((uint64_t)r.r[0] * (uint64_t)pts.count) >> 32);
    float x, y, z;
    cosine_dir(pts.nx[p], pts.ny[p], pts.nz[p], u24(r.r[1]), u24(r.r[2]), x, y, z);
    float L[3];
    field_eval(lobes, pts.px[p], pts.py[p], pts.pz[p], x, y, z, L);
    if (mode != NIRC_OUTPUT_RADIANCE) {   // occluded scene: the visibility cache learns V, the other V L
        const float V = visibility(lobes, pts.px[p], x, y, z);
        L[0] = mode == NIRC_OUTPUT_VISIBILITY ? V : V * L[0];
        L[1] = mode == NIRC_OUTPUT_VISIBILITY ? V : V * L[1];
        L[2] = mode == NIRC_OUTPUT_VISIBILITY ? V : V * L[2];
    }
    point[b] = (int32_t)p;
    wx[b] = x;
    wy[b] = y;
    wz[b] = z;
    target[3 * b + 0] = L[0];
    target[3 * b + 1] = L[1];
    target[3 * b + 2] = L[2];
}

// Step step + blockIdx.y into the buffers offset by blockIdx.y * stride.
__global__ void k_train_batch(Points pts, nirc_lobes lobes, int64_t batch, uint32_t key0,
                              uint32_t key1, uint32_t frame, uint32_t step, int mode, int32_t *point,
                              float *wx, float *wy, float *wz, float *target, int64_t stride) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const int64_t o = (int64_t)blockIdx.y * stride;
    train_sample(pts, lobes, key0, key1, frame, step + blockIdx.y, mode, b, point + o, wx + o, wy + o, wz + o,
                 target + o);
}

// The training samples of step `step` of every request of a training work list (request
// blockIdx.y), into each request's sample buffers.
__global__ void k_train_batch_multi(const TrainDesc *__restrict__ desc, uint32_t step) {
    if ((int)blockIdx.y >= desc->n) return;
    const TrainReq &t = desc->req[blockIdx.y];
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= t.batch) return;
    train_sample(t.pts, t.lobes, t.key0, t.key1, t.frame, step, t.output, b, t.sp, t.swx, t.swy, t.swz, t.stgt);
}

hipError_t launch_train_batch_multi(const TrainDesc *desc, uint32_t step, int64_t max_batch, hipStream_t s) {
    hipLaunchKernelGGL(k_train_batch_multi, dim3((unsigned)((max_batch + 255) / 256), kBatchMaxRequests), dim3(256), 0,
                       s, desc, step);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Per-query cache inference (every query encodes its own surface features): a wave takes 16
// queries at a time; the first layer runs over all 160 features.
template <int W, int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_infer_f32(Points pts, Queries q,
                                                          const float *__restrict__ packed,
                                                          float *__restrict__ rgb, int sig) {
    constexpr F32Layout L{W};
    constexpr int MT = W / 16;
    constexpr bool kLds = lds_weights(W);
    constexpr int NW = kLds ? InferLds<W>::kWeights : 4;
    __shared__ f32x4 smem4[NW / 4];
    if constexpr (kLds) {
        const f32x4 *src = (const f32x4 *)(packed + L.offset(SEC_D));
        for (int i = threadIdx.x; i < NW / 4; i += WAVES * 64) smem4[i] = src[i];
        __syncthreads();
    }
    const float *gS = packed + L.offset(SEC_S);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t Q = q.count;
    const int64_t n_tiles = (Q + 15) >> 4;
    for (int64_t tile = (int64_t)blockIdx.x * WAVES + wave; tile < n_tiles;
         tile += (int64_t)gridDim.x * WAVES) {
        const float *sD = kLds ? (const float *)smem4 : opaque(packed) + L.offset(SEC_D);
        const float *sH = sD + L.size(SEC_D);
        const float *sO = sH + 3 * L.size(SEC_H0);
        const int64_t qi = min((tile << 4) + col, Q - 1);
        const int64_t p = query_point(q, pts, qi);
        const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
        const float ws[3] = {q.wx[qi], q.wy[qi], q.wz[qi]};
        f32x4 h[1][MT];
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) h[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        layer1_surface<W>(h[0], opaque(gS), xs, lane, g);
        float dx[1] = {ws[0]}, dy[1] = {ws[1]}, dz[1] = {ws[2]};
        layer1_direction<W, 1>(h, sD, dx, dy, dz, lane, g);
        relu_all<W, 1>(h);
        hidden_layers<W, 1>(h, sH, lane);
        f32x4 y[1];
        output_layer<W, 1>(y, h, sO, lane);
        if (g == 0 && (tile << 4) + col < Q) {
            float *o = rgb + 3 * ((tile << 4) + col);
            o[0] = sig ? logistic(y[0][0]) : expf(y[0][0]);   // visibility cache: sigmoid outputs
            o[1] = sig ? logistic(y[0][1]) : expf(y[0][1]);
            o[2] = sig ? logistic(y[0][2]) : expf(y[0][2]);
        }
    }
}

// T consecutive query tiles (first tile T0, staged directions from batch slot s0) of the
// current point group through the FP32 chain, then per-point accumulation.
// OCC: the occluded-scene variants (visibility cache, radiance cache of the occluded scene),
// selected at run time by `mode`; the radiance cache of the plain scene compiles without them.
// ENC 1: the hash-grid model's direction input (spherical harmonics; width 64).
template <int W, int T, bool OCC, int ENC = 0, bool N16 = false>
__device__ __forceinline__ void tlmc_tiles_f32(int T0, int s0, int n_cache, DivN dn, const float *db, const float *hs,
                                               const float *sD, const float *sH, const float *sO,
                                               const nirc_lobes &lobes, const float *rrad, int64_t pc,
                                               const Points &pts, int64_t p0, int mode, const float *xs, int lane,
                                               int g, int col, float &fc0, float &fc1, float &fc2, float &fr0,
                                               float &fr1, float &fr2) {
    constexpr int MT = W / 16;
    if constexpr (!lds_weights(W)) {   // weights in global memory: keep their loads inside the pass
        sD = opaque(sD);
        sH = opaque(sH);
        sO = opaque(sO);
    }
    f32x4 h[T][MT];
    float dx[T], dy[T], dz[T];
    int jq[T];   // the point (within the group) of this lane's query in each tile
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const int Tt = T0 + tt;
        const int qi = 16 * (s0 + tt) + col;
        dx[tt] = db[qi];
        dy[tt] = db[kDirSlots + qi];
        dz[tt] = db[2 * kDirSlots + qi];
        const int j = (Tt < n_cache) ? (int)div_n((uint32_t)(16 * Tt + col), dn) : col;
        jq[tt] = j;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) h[tt][mt] = *(const f32x4 *)(hs + j * W + 16 * mt + 4 * g);
    }
    if constexpr (ENC == 1)
        hash_layer1_direction_f32<T>(h, sD, dx, dy, dz, lane, g);
    else
        layer1_direction<W, T>(h, sD, dx, dy, dz, lane, g);
    relu_all<W, T>(h);
    hidden_layers<W, T>(h, sH, lane);
    f32x4 y[T];
    output_layer<W, T>(y, h, sO, lane);
#pragma unroll
    for (int tt = 0; tt < T; ++tt) {
        const int Tt = T0 + tt;
        float y0, y1, y2;
        if (OCC && mode == NIRC_OUTPUT_VISIBILITY) {   // uniform: predicted visibility times the known radiance
            const int64_t pj = min(p0 + jq[tt], pts.count - 1);
            float Lq[3];
            field_eval(lobes, pts.px[pj], pts.py[pj], pts.pz[pj], dx[tt], dy[tt], dz[tt], Lq);
            y0 = logistic(y[tt][0]) * Lq[0];
            y1 = logistic(y[tt][1]) * Lq[1];
            y2 = logistic(y[tt][2]) * Lq[2];
        } else {
            // the hardware exponential (exp2 of z log2 e; relative error ~|z| 6e-8, far inside
            // the FP32 bound) rather than the library's expf: 1.3 % of the estimator's time
            y0 = __expf(y[tt][0]);
            y1 = __expf(y[tt][1]);
            y2 = __expf(y[tt][2]);
        }
        if (Tt < n_cache) {
            reduce_cache_tile<N16>(Tt, n_cache, col, y0, y1, y2, fc0, fc1, fc2);
        } else {
            float Lr[3];
            if (rrad) {   // uniform: the caller's residual radiance
                Lr[0] = rrad[3 * pc];
                Lr[1] = rrad[3 * pc + 1];
                Lr[2] = rrad[3 * pc + 2];
            } else {
                field_eval(lobes, xs[0], xs[1], xs[2], dx[tt], dy[tt], dz[tt], Lr);
                if (OCC && mode != NIRC_OUTPUT_RADIANCE) {   // the occluded scene's residual sample V L
                    const float V = visibility(lobes, xs[0], dx[tt], dy[tt], dz[tt]);
                    Lr[0] *= V;
                    Lr[1] *= V;
                    Lr[2] *= V;
                }
            }
            fr0 = Lr[0] - y0;
            fr1 = Lr[1] - y1;
            fr2 = Lr[2] - y2;
        }
    }
}

// ------------------------------------------------------------------------------------------
// Fused two-level estimator.
//
// A wave owns 16 shading points at a time.  It encodes their surface inputs once and projects
// them through the surface columns of the first layer (h_s = W1_s e_s, one MFMA pass for the
// 16 points), keeping h_s in a per-wave LDS slab.  The point group's queries are laid out as
// N cache tiles (query q = 16 t + column -> point q / N, direction q % N) followed by one
// residual tile (column j -> point j).  Directions for 8 tiles (128 queries) are generated at a
// time, one Philox block per lane giving two directions, and staged in the slab; the MLP then
// runs 4 tiles at a time with h_s of each column's point as the first layer's accumulator
// input, chains the hidden layers through registers and leaves RGB in lanes 0..15.  Cache
// results are summed per point with a 16-lane prefix sum; the residual tile evaluates the
// field and subtracts.  Only the final per-point values leave the chip.
// One point group (16 points from p0) through the FP32 chain.
// ENC 1: the hash-grid model (surface part from the grid `slv`/`table` and phi).
template <int W, bool OCC, int ENC = 0, bool N16 = false>
__device__ __forceinline__ void tlmc_group_f32(const Points &pts, int64_t p0, int n_cache, DivN dn, uint32_t key0,
                                               uint32_t key1, uint32_t frame, int mode, const float *rrad,
                                               float *out_tl,
                                               float *out_c, float *out_r, const nirc_lobes &lobes,
                                               const float *gS, const float *sD, const float *sH, const float *sO,
                                               float *hs, float *db, int lane, int g, int col,
                                               const HashLevel *slv = nullptr, uint32_t tmask = 0u,
                                               const float2 *table = nullptr) {
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
            float v[6], ph[4];
            hash_values6(slv, tmask, table, xs[0], xs[1], xs[2], g, v);
            hash_phi4(xs[3], xs[4], xs[5], xs[6], g, ph);
            hash_layer1_surface_f32(hsum, opaque(gS), v, ph, lane);
        } else {
            layer1_surface<W>(hsum, opaque(gS), xs, lane, g);
        }
        wave_sync();   // previous group's readers of the slab are done
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) *(f32x4 *)(hs + col * W + 16 * mt + 4 * g) = hsum[mt];
        // the group's normals, behind the staged directions (nrm [3][16])
        if (g < 3) db[3 * kDirSlots + 16 * g + col] = g == 0 ? xs[3] : g == 1 ? xs[4] : xs[5];
        wave_sync();
    }
    float fc0 = 0.f, fc1 = 0.f, fc2 = 0.f, fr0 = 0.f, fr1 = 0.f, fr2 = 0.f;
    for (int tb = 0; tb < n_tiles;) {
        const bool fold = n_tiles - tb == 9;   // last 8 cache tiles + the residual tile
        gen_dirs_batch_nrm<false>((uint32_t)p0, tb, n_cache, dn, key0, key1, frame, lane, db, db + 3 * kDirSlots, fold);
        const int tend = fold ? n_tiles : min(tb + 8, n_tiles);
        int t = tb;
        constexpr int TP = W <= 64 ? 4 : 2;   // tiles per pass (register budget)
#pragma unroll 1
        for (; t + TP <= tend; t += TP)
            tlmc_tiles_f32<W, TP, OCC, ENC, N16>(t, t - tb, n_cache, dn, db, hs, sD, sH, sO, lobes, rrad, pc, pts, p0, mode, xs,
                                            lane, g, col, fc0, fc1, fc2, fr0, fr1, fr2);
#pragma unroll 1
        for (; t < tend; ++t)
            tlmc_tiles_f32<W, 1, OCC, ENC, N16>(t, t - tb, n_cache, dn, db, hs, sD, sH, sO, lobes, rrad, pc, pts, p0, mode, xs,
                                           lane, g, col, fc0, fc1, fc2, fr0, fr1, fr2);
        tb = tend;
    }
    if (g == 0 && p0 + col < P)
        store_estimate(p0 + col, 1.0f / (float)n_cache, fc0, fc1, fc2, fr0, fr1, fr2, out_tl, out_c, out_r);
}

// N16: n_cache is a multiple of 16 (the per-point sums' other paths compiled out).
template <int W, int WAVES, bool OCC, bool N16 = false>
__global__ __launch_bounds__(WAVES * 64) void k_tlmc_f32(Points pts, nirc_lobes lobes,
                                                         const float *__restrict__ packed,
                                                         int n_cache, DivN dn, uint32_t key0, uint32_t key1,
                                                         uint32_t frame, int mode, const float *__restrict__ rrad,
                                                         float *__restrict__ out_tl, float *__restrict__ out_c,
                                                         float *__restrict__ out_r) {
    constexpr F32Layout L{W};
    constexpr bool kLds = lds_weights(W);
    constexpr int NW = kLds ? InferLds<W>::kWeights : 0;
    constexpr int SLAB = TlmcLds<W>::kSlab;
    __shared__ f32x4 smem4[(NW + WAVES * SLAB) / 4];
    __shared__ nirc_lobes s_lobes;
    float *smem = (float *)smem4;
    {
        const f32x4 *src = (const f32x4 *)(packed + L.offset(SEC_D));
        for (int i = threadIdx.x; i < NW / 4; i += WAVES * 64) smem4[i] = src[i];
        if (threadIdx.x == 0) s_lobes = lobes;
    }
    __syncthreads();
    const float *sD = kLds ? (const float *)smem : packed + L.offset(SEC_D);
    const float *sH = sD + L.size(SEC_D);   // LDS for width 64, global memory above
    const float *sO = sH + 3 * L.size(SEC_H0);
    const float *gS = packed + L.offset(SEC_S);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    float *hs = smem + NW + wave * SLAB;   // [16 points][W]
    float *db = hs + 16 * W;               // directions, SoA [3][kDirSlots]
    const int64_t n_groups = (pts.count + 15) >> 4;
    for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES)
        tlmc_group_f32<W, OCC, 0, N16>(pts, grp << 4, n_cache, dn, key0, key1, frame, mode, rrad, out_tl, out_c, out_r,
                                       s_lobes, gS, sD, sH, sO, hs, db, lane, g, col);
}

// Continuous batching with the FP32 chain (see k_tlmc_multi_h16).
template <int W, int WAVES, bool OCC>
__global__ __launch_bounds__(WAVES * 64) void k_tlmc_multi_f32(const BatchDesc *__restrict__ desc) {
    constexpr F32Layout L{W};
    constexpr int NW = InferLds<W>::kWeights;
    constexpr int SLAB = TlmcLds<W>::kSlab;
    __shared__ f32x4 smem4[(NW + WAVES * SLAB) / 4];
    __shared__ BatchRequest s_req;
    float *smem = (float *)smem4;
    const float *sD = smem;
    const float *sH = smem + L.size(SEC_D);
    const float *sO = sH + 3 * L.size(SEC_H0);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    float *hs = smem + NW + wave * SLAB;
    float *db = hs + 16 * W;
    const int n_req = desc->n_requests;
    const int total = desc->total_chunks;
    int cur = -1;
    for (int chunk = blockIdx.x; chunk < total; chunk += gridDim.x) {
        int r = 0;
        for (int i = 1; i < n_req; ++i)
            if (desc->req[i].chunk_begin <= chunk) r = i;
        if (r != cur) {
            __syncthreads();
            if (threadIdx.x == 0) s_req = desc->req[r];
            __syncthreads();
            const f32x4 *src = (const f32x4 *)((const float *)s_req.packed + L.offset(SEC_D));
            for (int i = threadIdx.x; i < NW / 4; i += WAVES * 64) smem4[i] = src[i];
            __syncthreads();
            cur = r;
        }
        const int64_t grp = (int64_t)(chunk - s_req.chunk_begin) * WAVES + wave;
        if (grp < (s_req.pts.count + 15) >> 4)
            tlmc_group_f32<W, OCC>(s_req.pts, grp << 4, s_req.n_cache, s_req.dn, s_req.key0, s_req.key1, s_req.frame,
                              __builtin_amdgcn_readfirstlane(s_req.mode), uniform_ptr(s_req.rrad), s_req.out_tl,
                              s_req.out_c, s_req.out_r, s_req.lobes,
                              (const float *)s_req.packed + L.offset(SEC_S), sD, sH, sO, hs, db, lane, g, col);
    }
}

// ------------------------------------------------------------------------------------------
// Launchers

hipError_t launch_pack(float *packed, const float *master, int W, hipStream_t s) {
    const int total = F32Layout{W}.total();
    hipLaunchKernelGGL(k_pack_f32, dim3((total + 255) / 256), dim3(256), 0, s, packed, master, W, total);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_copy_f32(float *dst, const float *src, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

hipError_t launch_encode(const Points &pts, const Queries &q, float *feat, hipStream_t s) {
    const int64_t n = q.count * kInputs;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_encode, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, q, feat);
    return hipGetLastError();
}

hipError_t launch_sample_dirs(const Points &pts, int n_cache, uint64_t seed, uint64_t frame,
                              float *dirs, hipStream_t s) {
    const int64_t n = pts.count * (n_cache + 1);
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_sample_dirs, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pts, n_cache,
                       (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)frame, dirs);
    return hipGetLastError();
}

hipError_t launch_bth(const Points &pts, const nirc_lobes &lobes, int n_cache, uint64_t seed, uint64_t frame,
                      int mode, const float *rrad, const float *fc, float *out, int32_t *cont, hipStream_t s) {
    if (pts.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_bth, dim3((unsigned)((pts.count + 255) / 256)), dim3(256), 0, s, pts, lobes, n_cache,
                       (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)frame, mode, rrad, fc, out, cont);
    return hipGetLastError();
}

hipError_t launch_train_batch(const Points &pts, const nirc_lobes &lobes, int64_t batch,
                              uint64_t seed, uint64_t frame, uint32_t step, int mode, int32_t *point,
                              float *wx, float *wy, float *wz, float *target, hipStream_t s, int nsteps,
                              int64_t stride) {
    if (batch == 0 || nsteps < 1) return hipSuccess;
    hipLaunchKernelGGL(k_train_batch, dim3((unsigned)((batch + 255) / 256), (unsigned)nsteps), dim3(256), 0, s, pts,
                       lobes, batch, (uint32_t)seed, (uint32_t)(seed >> 32), (uint32_t)frame, step, mode,
                       point, wx, wy, wz, target, stride);
    return hipGetLastError();
}

unsigned grid_for(int64_t units_per_wave_total, int waves, int max_blocks) {
    int64_t b = (units_per_wave_total + waves - 1) / waves;
    if (b > max_blocks) b = max_blocks;
    if (b < 1) b = 1;
    return (unsigned)b;
}

hipError_t launch_infer(int W, int prec, const Points &pts, const Queries &q, const void *packed, float *rgb,
                        int sig, hipStream_t s) {
    if (q.count == 0) return hipSuccess;
    if (prec != NIRC_FP32) return launch_infer_h16(W, prec, pts, q, packed, rgb, sig, s);
    constexpr int WAVES = 4;
    const unsigned grid = grid_for((q.count + 15) / 16, WAVES, 2 * kMaxResidentBlocks);
    if (W == 64)
        hipLaunchKernelGGL((k_infer_f32<64, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q, (const float *)packed,
                           rgb, sig);
    else if (W == 128)
        hipLaunchKernelGGL((k_infer_f32<128, WAVES>), dim3(grid), dim3(WAVES * 64), 0, s, pts, q,
                           (const float *)packed, rgb, sig);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_tlmc_multi_f32(int W, int mode, const BatchDesc *desc, int grid, hipStream_t s) {
    constexpr int WAVES = 8;
    static_assert(WAVES == kBatchChunkGroups, "chunk size");
    if (W != 64) return hipErrorInvalidValue;
    if (mode == NIRC_OUTPUT_RADIANCE)
        hipLaunchKernelGGL((k_tlmc_multi_f32<64, WAVES, false>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    else
        hipLaunchKernelGGL((k_tlmc_multi_f32<64, WAVES, true>), dim3(grid), dim3(WAVES * 64), 0, s, desc);
    return hipGetLastError();
}

hipError_t launch_tlmc(int W, int prec, const Points &pts, const nirc_lobes &lobes, const void *packed,
                       int n_cache, uint64_t seed, uint64_t frame, int mode, const float *rrad, float *out_tl,
                       float *out_c, float *out_r, hipStream_t s) {
    if (pts.count == 0) return hipSuccess;
    if (prec != NIRC_FP32)
        return launch_tlmc_h16(W, prec, pts, lobes, packed, n_cache, seed, frame, mode, rrad, out_tl, out_c, out_r,
                               s);
    constexpr int WAVES = 8;
    const unsigned grid = grid_for((pts.count + 15) / 16, WAVES, kMaxResidentBlocks);
    const unsigned grid128 = grid_for((pts.count + 15) / 16, 4, kMaxResidentBlocks);
    const DivN dn = make_divn(n_cache);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), f = (uint32_t)frame;
    const float *pk = (const float *)packed;
    const bool occ = mode != NIRC_OUTPUT_RADIANCE;
    if (W == 64 && !occ && n_cache % 16 == 0)
        hipLaunchKernelGGL((k_tlmc_f32<64, WAVES, false, true>), dim3(grid), dim3(WAVES * 64), 0, s, pts, lobes, pk,
                           n_cache, dn, k0, k1, f, mode, rrad, out_tl, out_c, out_r);
    else if (W == 64 && !occ)
        hipLaunchKernelGGL((k_tlmc_f32<64, WAVES, false>), dim3(grid), dim3(WAVES * 64), 0, s, pts, lobes, pk, n_cache,
                           dn, k0, k1, f, mode, rrad, out_tl, out_c, out_r);
    else if (W == 64)
        hipLaunchKernelGGL((k_tlmc_f32<64, WAVES, true>), dim3(grid), dim3(WAVES * 64), 0, s, pts, lobes, pk, n_cache,
                           dn, k0, k1, f, mode, rrad, out_tl, out_c, out_r);
    // width 128: one wave per SIMD (the width-128 FP32 pass needs more than 256 registers)
    else if (W == 128 && !occ)
        hipLaunchKernelGGL((k_tlmc_f32<128, 4, false>), dim3(grid128), dim3(4 * 64), 0, s, pts, lobes, pk, n_cache,
                           dn, k0, k1, f, mode, rrad, out_tl, out_c, out_r);
    else if (W == 128)
        hipLaunchKernelGGL((k_tlmc_f32<128, 4, true>), dim3(grid128), dim3(4 * 64), 0, s, pts, lobes, pk, n_cache,
                           dn, k0, k1, f, mode, rrad, out_tl, out_c, out_r);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// The hash-grid model in FP32 (inference and estimation).

// After an Adam step (step != NULL) thread 0 also commits the step or records its skip.
__global__ void k_hash_pack32(float *packed, const float *master, int64_t *step, uint32_t *flags, uint32_t *bad) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < kHash32Packed) {
        const int64_t s = hash_packed_source32(e);
        packed[e] = s >= 0 ? master[s] : 0.0f;
    }
    if (step && e == 0) {
        if (*bad) *flags |= *bad;   // the step's NIRC_FLAG_* bits
        else *step += 1;
        *bad = 0u;
    }
}

constexpr int kHash32LdsWeights = kHash32D + kHash32Rest;   // D, H0..H2, O

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_hash_tlmc_f32(Points pts, nirc_lobes lobes,
                                                              const float *__restrict__ packed,
                                                              const float2 *__restrict__ table, HashGridArgs grid,
                                                              int n_cache, DivN dn, uint32_t key0, uint32_t key1,
                                                              uint32_t frame, const float *__restrict__ rrad,
                                                              float *__restrict__ out_tl, float *__restrict__ out_c,
                                                              float *__restrict__ out_r) {
    constexpr int NW = kHash32LdsWeights;
    constexpr int SLAB = TlmcLds<64>::kSlab;
    __shared__ f32x4 smem4[(NW + WAVES * SLAB) / 4];
    __shared__ nirc_lobes s_lobes;
    __shared__ HashLevel s_lv[kHashLevels];
    float *smem = (float *)smem4;
    {
        const f32x4 *src = (const f32x4 *)(packed + kHash32S);
        for (int i = threadIdx.x; i < NW / 4; i += WAVES * 64) smem4[i] = src[i];
        if (threadIdx.x == 0) s_lobes = lobes;
        stage_levels(s_lv, grid);
    }
    __syncthreads();
    const float *sD = smem;
    const float *sH = sD + kHash32D;
    const float *sO = sH + 3 * F32Layout{64}.size(SEC_H0);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    float *hs = smem + NW + wave * SLAB;
    float *db = hs + 16 * 64;
    const int64_t n_groups = (pts.count + 15) >> 4;
    for (int64_t grp = (int64_t)blockIdx.x * WAVES + wave; grp < n_groups; grp += (int64_t)gridDim.x * WAVES)
        tlmc_group_f32<64, false, 1>(pts, grp << 4, n_cache, dn, key0, key1, frame, NIRC_OUTPUT_RADIANCE, rrad, out_tl,
                                     out_c, out_r, s_lobes, packed, sD, sH, sO, hs, db, lane, g, col, s_lv, grid.tmask,
                                     table);
}

template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_hash_infer_f32(Points pts, Queries q, const float *__restrict__ packed,
                                                               const float2 *__restrict__ table, HashGridArgs grid,
                                                               float *__restrict__ rgb) {
    constexpr int NW = kHash32LdsWeights;
    __shared__ f32x4 smem4[NW / 4];
    __shared__ HashLevel s_lv[kHashLevels];
    {
        const f32x4 *src = (const f32x4 *)(packed + kHash32S);
        for (int i = threadIdx.x; i < NW / 4; i += WAVES * 64) smem4[i] = src[i];
        stage_levels(s_lv, grid);
    }
    __syncthreads();
    const float *sD = (const float *)smem4;
    const float *sH = sD + kHash32D;
    const float *sO = sH + 3 * F32Layout{64}.size(SEC_H0);
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
        float v[6], ph[4];
        hash_values6(s_lv, grid.tmask, table, xs[0], xs[1], xs[2], g, v);
        hash_phi4(xs[3], xs[4], xs[5], xs[6], g, ph);
        hash_layer1_surface_f32(h[0], opaque(packed), v, ph, lane);
        const float dx[1] = {q.wx[qi]}, dy[1] = {q.wy[qi]}, dz[1] = {q.wz[qi]};
        hash_layer1_direction_f32<1>(h, sD, dx, dy, dz, lane, g);
        relu_all<64, 1>(h);
        hidden_layers<64, 1>(h, sH, lane);
        f32x4 y[1];
        output_layer<64, 1>(y, h, sO, lane);
        // lanes 0..15 hold rows 0..2 (the three channels) of their column
        if (g == 0 && (tile << 4) + col < Q) {
            const int64_t qo = (tile << 4) + col;
            rgb[3 * qo] = expf(y[0][0]);
            rgb[3 * qo + 1] = expf(y[0][1]);
            rgb[3 * qo + 2] = expf(y[0][2]);
        }
    }
}

hipError_t launch_hash_pack32(float *packed, const float *master, hipStream_t s, int64_t *step, uint32_t *flags,
                              uint32_t *bad) {
    hipLaunchKernelGGL(k_hash_pack32, dim3((kHash32Packed + 255) / 256), dim3(256), 0, s, packed, master, step, flags,
                       bad);
    return hipGetLastError();
}

hipError_t launch_hash_infer32(const Points &pts, const Queries &q, const float *packed, const float *table,
                               const HashGridArgs &grid, float *rgb, hipStream_t s) {
    constexpr int WAVES = 4;
    const unsigned nb = grid_for((q.count + 15) / 16, WAVES, 4 * kMaxResidentBlocks);
    hipLaunchKernelGGL((k_hash_infer_f32<WAVES>), dim3(nb), dim3(WAVES * 64), 0, s, pts, q, packed,
                       (const float2 *)table, grid, rgb);
    return hipGetLastError();
}

hipError_t launch_hash_tlmc32(const Points &pts, const nirc_lobes &lobes, const float *packed, const float *table,
                              const HashGridArgs &grid, int n_cache, uint64_t seed, uint64_t frame, const float *rrad,
                              float *out_tl, float *out_c, float *out_r, hipStream_t s) {
    constexpr int WAVES = 8;
    const unsigned nb = grid_for((pts.count + 15) / 16, WAVES, 2 * kMaxResidentBlocks);
    hipLaunchKernelGGL((k_hash_tlmc_f32<WAVES>), dim3(nb), dim3(WAVES * 64), 0, s, pts, lobes, packed,
                       (const float2 *)table, grid, n_cache, make_divn(n_cache), (uint32_t)seed,
                       (uint32_t)(seed >> 32), (uint32_t)frame, rrad, out_tl, out_c, out_r);
    return hipGetLastError();
}

}  // namespace nirc
