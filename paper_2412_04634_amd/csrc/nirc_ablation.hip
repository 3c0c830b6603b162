// The fused estimator's pipeline with its fusions undone, for measuring what each one buys (Sec.
// "Neural Network Architecture": the inference-pipeline comparison of shared surface encodings,
// the direction encoding fused into the network's first layer, and output written straight from
// on-chip memory).  16-bit models of width 64.  Stages, each a complete estimator:
//   0  every query's encoded inputs (surface and direction, 160 features as 16-bit MFMA operands)
//      are written to memory by one kernel and read back by the network kernel, which writes one
//      prediction per query; a third kernel reduces them per point and forms the residual;
//   1  as 0, with the surface inputs encoded once per point and shared by its N + 1 queries;
//   2  as 1, with the direction sampling and encoding done inside the network kernel;
//   3  the fused estimator (tlmc_estimate): surface projection once per point, directions and
//      their encoding in the kernel, per-point sums on chip, one store per point.
// Directions, features and arithmetic are those of the fused kernel, so every stage computes the
// same estimate up to the order of its sums.
#include "nirc_h16.hpp"

namespace nirc {

namespace {

constexpr int kAbWaves = 8;

// Query q of the unfused stages: point q / (N + 1), sample k = q % (N + 1) (k = N: residual).
__device__ __forceinline__ void query_of(uint32_t q, uint32_t n1, uint32_t &p, uint32_t &k) {
    p = q / n1;
    k = q - p * n1;
}

// The direction of sample k of point p, as the fused estimator draws it: cache directions with
// the hardware sine, the residual direction with the exact map.
__device__ __forceinline__ void sample_direction(const Points &pts, uint32_t p, uint32_t k, int n_cache, uint32_t key0,
                                                 uint32_t key1, uint32_t frame, float &wx, float &wy, float &wz) {
    const bool res = (int)k == n_cache;
    const DirCounter c = dir_counter(p, (int)k, res);
    const Rand4 r = philox(c.c0, c.c1, frame, c.stream, key0, key1);
    const float u1 = u24(c.half ? r.r[2] : r.r[0]), u2 = u24(c.half ? r.r[3] : r.r[1]);
    const float nx = pts.nx[p], ny = pts.ny[p], nz = pts.nz[p];
    if (res) {
        cosine_dir(nx, ny, nz, u1, u2, wx, wy, wz);
        return;
    }
    cosine_dir_fast(nx, ny, nz, u1, u2, wx, wy, wz);
}

// The surface features of lane group g (frequencies 2g, 2g + 1 of the 7 surface inputs) as the
// four B operands of the first layer's surface section.
template <int PREC>
__device__ __forceinline__ void surface_operands16(const Points &pts, uint32_t p, int g, u32x4 (&b)[4]) {
    const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
    float f[32];
#pragma unroll
    for (int i = 0; i < 7; ++i) enc_pair2_fast(xs[i], g, f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
    f[28] = f[29] = f[30] = f[31] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb)
        b[kb] = u32x4{pack2<PREC>(f[8 * kb], f[8 * kb + 1]), pack2<PREC>(f[8 * kb + 2], f[8 * kb + 3]),
                      pack2<PREC>(f[8 * kb + 4], f[8 * kb + 5]), pack2<PREC>(f[8 * kb + 6], f[8 * kb + 7])};
}

// The direction operands of lane group g exactly as the fused kernel builds them (all eight
// frequencies by angle doubling, dir_features16), of which lane group g takes 2g and 2g + 1.
template <int PREC>
__device__ __forceinline__ void direction_operands_chain(float dx, float dy, float dz, int g, u32x4 &b0, u32x4 &b1) {
    uint32_t px[8], py[8], pz[8];
    chain8<PREC>(dx, px);
    chain8<PREC>(dy, py);
    chain8<PREC>(dz, pz);
    b0 = u32x4{px[0], px[1], py[0], py[1]};
    b1 = u32x4{pz[0], pz[1], 0u, 0u};
#pragma unroll
    for (int gg = 1; gg < 4; ++gg)
        if (g == gg) {
            b0 = u32x4{px[2 * gg], px[2 * gg + 1], py[2 * gg], py[2 * gg + 1]};
            b1 = u32x4{pz[2 * gg], pz[2 * gg + 1], 0u, 0u};
        }
}

}  // namespace

// Stage 0: all six operands of each query ([tile][6][64 lanes] u32x4: surface K-blocks 0..3, then
// direction K-blocks 0..1).  Stage 1: the two direction operands only ([tile][2][64]).  One thread
// per (query, lane group).
template <int PREC>
__global__ __launch_bounds__(256) void k_ab_encode(Points pts, int n_cache, uint32_t key0, uint32_t key1,
                                                   uint32_t frame, int stage, int64_t Q, u32x4 *__restrict__ ops) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * Q) return;
    const uint32_t q = (uint32_t)(t >> 2);
    const int g = (int)(t & 3);
    uint32_t p, k;
    query_of(q, (uint32_t)n_cache + 1u, p, k);
    const uint32_t tile = q >> 4, lane = 16u * (uint32_t)g + (q & 15u);
    const int nk = stage == 0 ? 6 : 2;
    u32x4 *o = ops + (int64_t)tile * nk * 64 + lane;
    if (stage == 0) {
        u32x4 b[4];
        surface_operands16<PREC>(pts, p, g, b);
#pragma unroll
        for (int kb = 0; kb < 4; ++kb) o[kb * 64] = b[kb];
        o += 4 * 64;
    }
    float wx, wy, wz;
    sample_direction(pts, p, k, n_cache, key0, key1, frame, wx, wy, wz);
    u32x4 d0, d1;
    direction_operands_chain<PREC>(wx, wy, wz, g, d0, d1);
    o[0] = d0;
    o[64] = d1;
}

// Stages 1 and 2: the surface operands of each point ([point group][4][64 lanes] u32x4), one
// thread per (point, lane group).
template <int PREC>
__global__ __launch_bounds__(256) void k_ab_surface(Points pts, u32x4 *__restrict__ sops) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 4 * pts.count) return;
    const uint32_t p = (uint32_t)(t >> 2);
    const int g = (int)(t & 3);
    u32x4 b[4];
    surface_operands16<PREC>(pts, p, g, b);
    u32x4 *o = sops + (int64_t)(p >> 4) * 4 * 64 + 16 * g + (p & 15u);
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) o[kb * 64] = b[kb];
}

// The network over query tiles, four tiles per pass with the fused kernel's chain (weights of the
// direction, hidden and output sections staged in LDS; the surface section read from L2), inputs
// from memory (stages 0, 1: surface and direction operands; stage 2: surface operands, directions
// drawn and encoded here), one prediction per query written to y [Q][3].
template <int PREC, int STAGE>
__global__ __launch_bounds__(kAbWaves * 64) void k_ab_mlp(Points pts, const uint16_t *__restrict__ packed, int n_cache,
                                                          uint32_t key0, uint32_t key1, uint32_t frame, int64_t Q,
                                                          const u32x4 *__restrict__ qops,
                                                          const u32x4 *__restrict__ sops, float *__restrict__ y) {
    constexpr int W = 64, MT = 4, KB = 2, T = 4;
    constexpr H16Layout L{W};
    constexpr int NW = H16Layout{W}.offset(SEC_T0) - H16Layout{W}.offset(SEC_D);
    __shared__ u32x4 wsm[NW / 8];
    {
        const u32x4 *src = (const u32x4 *)(packed + L.offset(SEC_D));
        for (int i = threadIdx.x; i < NW / 8; i += kAbWaves * 64) wsm[i] = src[i];
    }
    __syncthreads();
    const uint16_t *sD = (const uint16_t *)wsm;
    const uint16_t *sH = sD + L.size(SEC_D);
    const uint16_t *sOS = sH + 3 * L.size(SEC_H0) + L.size(SEC_O);
    const uint16_t *gS = packed + L.offset(SEC_S);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    // stage 2: per pass, lane l draws and encodes query l % 16 of tile l / 16 once (all eight
    // frequencies), and every lane group picks up its operands from this wave's slab
    __shared__ u32x4 sfa[STAGE == 2 ? kAbWaves * 4 * 64 : 1];
    __shared__ uint2 sfb[STAGE == 2 ? kAbWaves * 4 * 64 : 1];
    const int64_t n_tiles = (Q + 15) >> 4;
    const int64_t n_pass = (n_tiles + T - 1) / T;
    u32x4 dfrag[W / 8];
    load_dir_fragments<W>(dfrag, sD, lane);
    for (int64_t pass = (int64_t)blockIdx.x * kAbWaves + wave; pass < n_pass; pass += (int64_t)gridDim.x * kAbWaves) {
        f32x4 h[T][MT];
        u32x4 bd[T][2];
        if constexpr (STAGE == 2) {
            const int64_t tile = min(pass * T + g, n_tiles - 1);
            const uint32_t q = (uint32_t)min((tile << 4) + col, Q - 1);
            uint32_t p, k;
            query_of(q, (uint32_t)n_cache + 1u, p, k);
            float wx, wy, wz;
            sample_direction(pts, p, k, n_cache, key0, key1, frame, wx, wy, wz);
            const int e0 = wave * 256 + 64 * g + col;   // entry (tile g, lane group 0, query col)
            wave_lds_order();   // after the previous pass's reads
            dir_features16<PREC>(wx, wy, wz, sfa + e0, sfb + e0, 16);
            wave_lds_order();
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt) {
            const int64_t tile = min(pass * T + tt, n_tiles - 1);
            const uint32_t q = (uint32_t)min((tile << 4) + col, Q - 1);
            u32x4 bs[4];
            if constexpr (STAGE == 0) {
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) bs[kb] = qops[tile * 6 * 64 + kb * 64 + lane];
                bd[tt][0] = qops[tile * 6 * 64 + 4 * 64 + lane];
                bd[tt][1] = qops[tile * 6 * 64 + 5 * 64 + lane];
            } else {
                uint32_t p, k;
                query_of(q, (uint32_t)n_cache + 1u, p, k);
                const u32x4 *sp = sops + (int64_t)(p >> 4) * 4 * 64 + 16 * g + (p & 15u);
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) bs[kb] = sp[kb * 64];
                if constexpr (STAGE == 1) {
                    bd[tt][0] = qops[tile * 2 * 64 + lane];
                    bd[tt][1] = qops[tile * 2 * 64 + 64 + lane];
                } else {
                    const int e = wave * 256 + (tt * 4 + g) * 16 + col;
                    bd[tt][0] = sfa[e];
                    const uint2 b = sfb[e];
                    bd[tt][1] = u32x4{b.x, b.y, 0u, 0u};
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt) h[tt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
            const uint16_t *gs = opaque(gS);
#pragma unroll
            for (int kb = 0; kb < 4; ++kb)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    h[tt][mt] = mfma16<PREC>(*(const u32x4 *)(gs + ((mt * 4 + kb) * 64 + lane) * 8), bs[kb], h[tt][mt]);
        }
        u32x4 hb[T][KB];
        u32x4 aout[4 * KB];
        mlp16<W, PREC, T>(h, hb, bd, dfrag, sH, sOS, lane, aout);
        const f32x4 z = output16_packed<W, PREC, T>(hb, aout);
        // lane (g, col): tile col / 3, channel col % 3, queries 4g + i of that tile
        const int tt = col / 3, c = col - 3 * (col / 3);
        if (col < 3 * T) {
            const int64_t tile = pass * T + tt;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int64_t q = (tile << 4) + 4 * g + i;
                if (tile < n_tiles && q < Q) y[3 * q + c] = __expf(z[i]);
            }
        }
    }
}

// Per point: F_c = mean of its N cache predictions (in sample order), F_r = L(x, w_r) - y(x, w_r)
// with the residual direction drawn again, F_tl = F_c + F_r.  A block of 64 points first copies
// their predictions (one contiguous run of 64 (N + 1) 3 floats) to LDS with coalesced loads when
// the run fits (N <= 63), then each thread sums its own point's row from there.
constexpr int kAbReduceRun = 64 * 64 * 3;   // floats (48 KB): the largest run staged
__global__ __launch_bounds__(64) void k_ab_reduce(Points pts, nirc_lobes lobes, int n_cache, uint32_t key0,
                                                  uint32_t key1, uint32_t frame, const float *__restrict__ y,
                                                  float *__restrict__ out_tl, float *__restrict__ out_c,
                                                  float *__restrict__ out_r) {
    extern __shared__ float run[];   // 64 (N + 1) 3 floats when staged (launch-time size)
    const int64_t p0 = (int64_t)blockIdx.x * 64, p = p0 + threadIdx.x;
    const int row = 3 * (n_cache + 1);
    const int64_t npts = min((int64_t)64, pts.count - p0);
    const bool staged = 64 * row <= kAbReduceRun;
    if (staged) {
        const float *src = y + p0 * row;
        for (int i = threadIdx.x; i < npts * row; i += 64) run[i] = src[i];
        __syncthreads();
    }
    if (p >= pts.count) return;
    const float *yp = staged ? run + threadIdx.x * row : y + p * row;
    float s[3] = {0.f, 0.f, 0.f};
    for (int k = 0; k < n_cache; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) s[c] += yp[3 * k + c];
    float wx, wy, wz;
    sample_direction(pts, (uint32_t)p, (uint32_t)n_cache, n_cache, key0, key1, frame, wx, wy, wz);
    float L[3];
    field_eval(lobes, pts.px[p], pts.py[p], pts.pz[p], wx, wy, wz, L);
    const float inv_n = 1.0f / (float)n_cache;
    store_estimate(p, inv_n, s[0], s[1], s[2], L[0] - yp[3 * n_cache], L[1] - yp[3 * n_cache + 1],
                   L[2] - yp[3 * n_cache + 2], out_tl, out_c, out_r);
}

// Workspace: y [Q][3] FP32, then the operand buffers of the stage.
struct AbLayout {
    size_t y, qops, sops, total;
    AbLayout(int64_t P, int n_cache, int stage) {
        const int64_t Q = P * (n_cache + 1), tiles = (Q + 15) / 16, groups = (P + 15) / 16;
        auto al = [](size_t x) { return (x + 255) / 256 * 256; };
        size_t o = 0;
        y = o;
        o += al((size_t)Q * 3 * sizeof(float));
        qops = o;
        o += stage == 0 ? al((size_t)tiles * 6 * 64 * 16) : stage == 1 ? al((size_t)tiles * 2 * 64 * 16) : 0;
        sops = o;
        o += (stage == 1 || stage == 2) ? al((size_t)groups * 4 * 64 * 16) : 0;
        total = o;
    }
};

size_t ablation_workspace_bytes(int64_t P, int n_cache, int stage) { return AbLayout(P, n_cache, stage).total; }

template <int PREC>
static hipError_t launch_ablation_t(int stage, const Points &pts, const nirc_lobes &lobes, const uint16_t *packed,
                                    int n_cache, uint64_t seed, uint64_t frame, char *ws, float *out_tl, float *out_c,
                                    float *out_r, hipStream_t s) {
    const AbLayout L(pts.count, n_cache, stage);
    const int64_t Q = pts.count * (n_cache + 1);
    const uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32), f = (uint32_t)frame;
    float *y = (float *)(ws + L.y);
    u32x4 *qops = (u32x4 *)(ws + L.qops), *sops = (u32x4 *)(ws + L.sops);
    if (stage <= 1)
        hipLaunchKernelGGL(k_ab_encode<PREC>, dim3((unsigned)((4 * Q + 255) / 256)), dim3(256), 0, s, pts, n_cache, k0,
                           k1, f, stage, Q, qops);
    if (stage >= 1)
        hipLaunchKernelGGL(k_ab_surface<PREC>, dim3((unsigned)((4 * pts.count + 255) / 256)), dim3(256), 0, s, pts,
                           sops);
    const dim3 grid(kMaxResidentBlocks), block(kAbWaves * 64);
    if (stage == 0)
        hipLaunchKernelGGL((k_ab_mlp<PREC, 0>), grid, block, 0, s, pts, packed, n_cache, k0, k1, f, Q, qops, sops, y);
    else if (stage == 1)
        hipLaunchKernelGGL((k_ab_mlp<PREC, 1>), grid, block, 0, s, pts, packed, n_cache, k0, k1, f, Q, qops, sops, y);
    else
        hipLaunchKernelGGL((k_ab_mlp<PREC, 2>), grid, block, 0, s, pts, packed, n_cache, k0, k1, f, Q, qops, sops, y);
    const int row = 3 * (n_cache + 1);
    const unsigned shmem = 64 * row <= kAbReduceRun ? (unsigned)(64 * row * sizeof(float)) : 0u;
    hipLaunchKernelGGL(k_ab_reduce, dim3((unsigned)((pts.count + 63) / 64)), dim3(64), shmem, s, pts, lobes, n_cache,
                       k0, k1, f, y, out_tl, out_c, out_r);
    return hipGetLastError();
}

hipError_t launch_ablation(int prec, int stage, const Points &pts, const nirc_lobes &lobes, const uint16_t *packed,
                           int n_cache, uint64_t seed, uint64_t frame, char *ws, float *out_tl, float *out_c,
                           float *out_r, hipStream_t s) {
    if (pts.count == 0) return hipSuccess;
    return prec == NIRC_BF16
               ? launch_ablation_t<NIRC_BF16>(stage, pts, lobes, packed, n_cache, seed, frame, ws, out_tl, out_c, out_r, s)
               : launch_ablation_t<NIRC_FP16>(stage, pts, lobes, packed, n_cache, seed, frame, ws, out_tl, out_c, out_r,
                                              s);
}

}  // namespace nirc
