// Device building blocks of the NIRC library for gfx950 (CDNA4): counter-based random numbers,
// cosine-weighted sampling, the sin/cos input encoding, MFMA wrappers and the packed weight
// layout that lets consecutive MLP layers chain through registers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nirc.h"

namespace nirc {

constexpr int kInputs = 10;
constexpr int kFreq = 8;
constexpr int kFeat = 160;
constexpr int kSurfInputs = 7;   // x0 x1 x2 n0 n1 n2 roughness
constexpr int kDirInputs = 3;    // w0 w1 w2
constexpr int kStreamCacheDir = 3, kStreamResidualDir = 4, kStreamTrain = 5, kStreamTerminate = 6;

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Canonical input index (x, w, n, roughness order) of surface input s.
__host__ __device__ constexpr int surf_input(int s) { return s < 3 ? s : s + 3; }

struct Points {
    const float *px, *py, *pz, *nx, *ny, *nz, *rough;
    int64_t count;
};

struct Queries {
    const float *wx, *wy, *wz;
    const int32_t *point;
    int64_t count;
    uint32_t *err;   // receives NIRC_FLAG_BAD_POINT_INDEX on an index out of range (nullable)
};

__device__ inline bool point_index_ok(const Queries &q, const Points &p, int64_t i) {
    if (!q.point) return true;
    const int64_t j = q.point[i];
    return j >= 0 && j < p.count;
}

// Point index of query i: explicit or i itself.  An explicit index outside [0, count) raises
// NIRC_FLAG_BAD_POINT_INDEX in q.err and is replaced by the nearest valid one, so that it never
// reads out of bounds; the outputs of such a query are not defined.
__device__ inline int64_t query_point(const Queries &q, const Points &p, int64_t i) {
    if (!q.point) return i;
    const int64_t j = q.point[i];
    if (j >= 0 && j < p.count) return j;
    if (q.err) atomicOr(q.err, NIRC_FLAG_BAD_POINT_INDEX);
    return j < 0 ? 0 : p.count - 1;
}

// Division of a query index q by the cache sample count N without a hardware divide:
// q / N = umulhi(q, ceil(2^32 / N)) exactly for q < 2^17 and 2 <= N <= 4096 (the rounding error
// q (M - 2^32/N) / 2^32 < 2^-15 stays below 1/N); N = 1 is the identity.
struct DivN {
    uint32_t n, magic;
};

__host__ inline DivN make_divn(int n) {
    DivN d;
    d.n = (uint32_t)n;
    d.magic = n <= 1 ? 0u : (uint32_t)((0x100000000ull + (uint64_t)n - 1) / (uint64_t)n);
    return d;
}

__device__ __forceinline__ uint32_t div_n(uint32_t q, DivN d) { return d.n == 1 ? q : __umulhi(q, d.magic); }

// ------------------------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): multiply-xor rounds on a 4x32 counter, key bumped by
// the Weyl constants between rounds.
struct Rand4 {
    uint32_t r[4];
};

__device__ inline Rand4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                               uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        if (round) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        // 32x32 -> 64-bit products (one v_mad_u64_u32 each)
        const uint64_t p0 = (uint64_t)c0 * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c2 * 0xCD9E8D57u;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c0 = n0;
        c1 = (uint32_t)p1;
        c2 = n2;
        c3 = (uint32_t)p0;
    }
    return Rand4{{c0, c1, c2, c3}};
}

// 24-bit uniform in [0, 1), exact in FP32.
__device__ inline float u24(uint32_t r) { return (float)(r >> 8) * 0x1p-24f; }

// sin and cos of 2 pi u for u in [0, 1) with at most 24 fractional bits (a 24-bit uniform).
// Octant reduction is exact: q = 8u, j = floor(q) and f = q - j carry no rounding, and the
// octant symmetries map the angle to x = g pi/4 with g = f (even j) or 1 - f (odd j), also
// exact.  On [0, pi/4] the Taylor series of sin to x^9 and of cos to x^10 truncate below
// 2e-9, so the pair is within a few ulp; the octant then swaps the two and sets their signs
// (swap for j = 1, 2, 5, 6; sin < 0 for j >= 4; cos < 0 for j = 2..5).
__host__ __device__ inline void sincos_turns(float u, float &s, float &c) {
#pragma clang fp contract(off)
    const float q = u * 8.0f;
    const float jf = floorf(q);
    const int j = (int)jf;
    const float f = q - jf;
    const float g = (j & 1) ? 1.0f - f : f;
    const float x = g * 0.785398163397448309616f;
    const float x2 = x * x;
    float sp = fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    sp = fmaf(x2, sp, 1.0f / 120.0f);
    sp = fmaf(x2, sp, -1.0f / 6.0f);
    const float sn = fmaf(x * x2, sp, x);
    float cp = fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    cp = fmaf(x2, cp, -1.0f / 720.0f);
    cp = fmaf(x2, cp, 1.0f / 24.0f);
    cp = fmaf(x2, cp, -0.5f);
    const float cs = fmaf(x2, cp, 1.0f);
    const bool swap = ((j + 1) >> 1) & 1;
    const float a = swap ? cs : sn, b = swap ? sn : cs;
    s = (j >= 4) ? -a : a;
    c = (((j + 2) >> 2) & 1) ? -b : b;
}

// sin(pi t) and cos(pi t) for |t| <= 2^22 (the encoding's arguments 2^k v, |v| <= 1, k <= 7):
// t = n/2 + r with n = rint(2t) and |r| <= 1/4, both exact; the Taylor series of sin (to x^9)
// and cos (to x^10) at x = pi r in [-pi/4, pi/4]; then the quarter turn n mod 4 swaps the pair and
// sets the signs.  Multiples of 1/2 give exact values; elsewhere a few ulp.
__host__ __device__ inline void sincospi_small(float t, float &s, float &c) {
#pragma clang fp contract(off)
    const float nf = rintf(2.0f * t);
    const float r = fmaf(nf, -0.5f, t);
    const float x = r * 3.14159265358979323846f;
    const float x2 = x * x;
    float sp = fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f);
    sp = fmaf(x2, sp, 1.0f / 120.0f);
    sp = fmaf(x2, sp, -1.0f / 6.0f);
    const float sn = fmaf(x * x2, sp, x);
    float cp = fmaf(x2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
    cp = fmaf(x2, cp, -1.0f / 720.0f);
    cp = fmaf(x2, cp, 1.0f / 24.0f);
    cp = fmaf(x2, cp, -0.5f);
    const float cs = fmaf(x2, cp, 1.0f);
    const int q = (int)nf & 3;
    const float a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// Cosine-weighted direction about unit normal n from uniforms (u1, u2): local
// (sqrt(u1) cos 2pi u2, sqrt(u1) sin 2pi u2, sqrt(1 - u1)) in the branchless orthonormal basis
// of Duff et al. (JCGT 2017).  sin/cos from sincos_turns, square roots and the reciprocal from
// the hardware instructions (1 ulp): the direction is within a few 1e-7 of the exact map.
// Contraction is off so that every kernel that inlines this produces bit-identical directions.
__device__ inline void cosine_dir(float nx, float ny, float nz, float u1, float u2, float &wx,
                                  float &wy, float &wz) {
#pragma clang fp contract(off)
    const float r = __builtin_amdgcn_sqrtf(u1);
    float s2, c2;
    sincos_turns(u2, s2, c2);
    const float lx = r * c2, ly = r * s2, lz = __builtin_amdgcn_sqrtf(1.0f - u1);
    const float s = nz >= 0.0f ? 1.0f : -1.0f;
    const float a = -__builtin_amdgcn_rcpf(s + nz);   // |s + nz| is in [1, 2]: no range issues
    const float b = nx * ny * a;
    const float tx = 1.0f + s * nx * nx * a, ty = s * b, tz = -s * nx;
    const float bx = b, by = s + ny * ny * a, bz = -ny;
    wx = lx * tx + ly * bx + lz * nx;
    wy = lx * ty + ly * by + lz * ny;
    wz = lx * tz + ly * bz + lz * nz;
}

// Philox counter of a sampled direction and which word pair it uses.  Cache direction k of
// point p: (p, k >> 1, frame, 3), pair k & 1.  Residual direction of p: (p >> 1, 0, frame, 4),
// pair p & 1.
struct DirCounter {
    uint32_t c0, c1;
    uint32_t stream;
    int half;
};

__device__ inline DirCounter dir_counter(uint32_t p, int k, bool residual) {
    if (residual) return DirCounter{p >> 1, 0u, (uint32_t)kStreamResidualDir, (int)(p & 1u)};
    return DirCounter{p, (uint32_t)k >> 1, (uint32_t)kStreamCacheDir, k & 1};
}

__device__ inline void dir_from_rand(const Rand4 &r, int half, float nx, float ny, float nz,
                                     float &wx, float &wy, float &wz) {
    const uint32_t a = half ? r.r[2] : r.r[0];
    const uint32_t b = half ? r.r[3] : r.r[1];
    cosine_dir(nx, ny, nz, u24(a), u24(b), wx, wy, wz);
}

// ------------------------------------------------------------------------------------------
// Radiance field (stand-in for path-traced radiance): sum of four spherical-Gaussian lobes
// with amplitudes linear in x.
__device__ inline void field_eval(const nirc_lobes &L, float x0, float x1, float x2, float wx,
                                  float wy, float wz, float out[3]) {
    out[0] = out[1] = out[2] = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float mw = L.axis[j][0] * wx + L.axis[j][1] * wy + L.axis[j][2] * wz;
        const float g = expf(L.kappa[j] * (mw - 1.0f));
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float a = L.alpha[j][c] + L.beta[j][c][0] * x0 + L.beta[j][c][1] * x1 +
                            L.beta[j][c][2] * x2;
            out[c] += a * g;
        }
    }
}

// Lobe j's contribution to the field (the terms of field_eval for one j).
__device__ inline void field_lobe(const nirc_lobes &L, int j, float x0, float x1, float x2, float wx, float wy,
                                  float wz, float out[3]) {
    const float mw = L.axis[j][0] * wx + L.axis[j][1] * wy + L.axis[j][2] * wz;
    const float gj = expf(L.kappa[j] * (mw - 1.0f));
#pragma unroll
    for (int c = 0; c < 3; ++c)
        out[c] = (L.alpha[j][c] + L.beta[j][c][0] * x0 + L.beta[j][c][1] * x1 + L.beta[j][c][2] * x2) * gj;
}

// Channel c of the field.
__device__ inline float field_channel(const nirc_lobes &L, int c, float x0, float x1, float x2, float wx, float wy,
                                      float wz) {
    float acc = 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float mw = L.axis[j][0] * wx + L.axis[j][1] * wy + L.axis[j][2] * wz;
        acc += (L.alpha[j][c] + L.beta[j][c][0] * x0 + L.beta[j][c][1] * x1 + L.beta[j][c][2] * x2) *
               expf(L.kappa[j] * (mw - 1.0f));
    }
    return acc;
}

// Synthetic visibility of the occluded (environment-lit) scene: a soft cap over the first lobe's
// axis mu_0 that blocks 90 % of it, V = 1 - 0.9 / (1 + exp(-16 (mu_0 . w - c(x)))) with
// c(x) = 0.6 + 0.3 (x_0 - 0.5).
__device__ inline float visibility(const nirc_lobes &L, float x0, float wx, float wy, float wz) {
    const float m = L.axis[0][0] * wx + L.axis[0][1] * wy + L.axis[0][2] * wz;
    const float c = 0.6f + 0.3f * (x0 - 0.5f);
    return 1.0f - 0.9f / (1.0f + expf(-16.0f * (m - c)));
}

__device__ inline float logistic(float z) { return 1.0f / (1.0f + expf(-z)); }

// ------------------------------------------------------------------------------------------
// MFMA wrappers (wave64).  16x16x4 FP32: lane l holds A[row l%16][k l/16], B[k l/16][col l%16];
// the 16x16 result gives lane l rows 4(l/16)+i, i = 0..3, of column l%16.
__device__ inline f32x4 mfma4(float a, float b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Exact-argument sin/cos(pi * 2^k * v): 2^k v is exact in FP32, sincospif reduces exactly.
__device__ inline void enc_pair(float v, int k, float &s, float &c) {
    sincospi_small(ldexpf(v, k), s, c);
}

// ReLU on the FP32 bits: a signed integer max with 0 maps every negative value (sign bit set)
// to +0 and leaves the rest unchanged, in one instruction (a float max must first quiet
// signalling NaNs, which doubles its cost).
__device__ __forceinline__ float relu_f32(float x) {
    const int v = __builtin_bit_cast(int, x);
    return __builtin_bit_cast(float, v > 0 ? v : 0);
}

// Frequencies k and k + 1: the exact pair at k, then one angle doubling (sin 2a = 2 sin a cos a,
// cos 2a = (cos a - sin a)(cos a + sin a)), within ~2 ulp of the exact pair at k + 1.
// Contraction is off so that every kernel that inlines this computes the same bits.
__device__ inline void enc_pair2(float v, int k, float &s0, float &c0, float &s1, float &c1) {
#pragma clang fp contract(off)
    enc_pair(v, k, s0, c0);
    s1 = 2.0f * (s0 * c0);
    c1 = (c0 - s0) * (c0 + s0);
}

// ------------------------------------------------------------------------------------------
// Packed weights for the FP32 MFMA chain.
//
// Each layer product is computed as H^T = W X^T with the weights as the MFMA A operand and the
// queries as the 16 columns of B.  The result leaves lane l with neurons 16m + 4(l/16) + i of
// query l%16 (m = row tile, i = 0..3).  Reading K-block b = 4m + i of the next layer as "lane
// group g holds neuron 16m + 4g + i" turns those registers into the next B operand with no data
// movement, provided the next layer's weight columns are permuted to match; the packed copy
// stores every layer's A fragments in that order:
//   fragment (mt, kb), lane l: row 16 mt + l%16, K position 4 kb + l/16,
//   stored at [mt][kb / 4][lane][kb % 4] so that one 16-byte LDS read fetches 4 K-blocks.
// Input features are produced directly in B layout: lane group g computes frequencies 2g and
// 2g+1 of every input, so its t-th feature (t = 4 i + 2 f + sc) is input i, frequency 2g + f,
// sin (sc = 0) or cos (sc = 1), placed in K-block t at position g.
//
// Sections (W = hidden width):
//   S   W1 surface columns    MT = W/16, KB = 28   (x0 x1 x2 n0 n1 n2 r)
//   D   W1 direction columns  MT = W/16, KB = 12   (w0 w1 w2)
//   H0..H2  W2, W3, W4        MT = W/16, KB = W/4
//   O   W5 (3 rows padded)    MT = 1,    KB = W/4
//   T0..T2  W2^T, W3^T, W4^T  MT = W/16, KB = W/4  (backward: delta_{l-1} = W_l^T delta_l)
//   OT  W5^T                  MT = W/16, KB = 4    (K = output rows padded to 16)
enum Section { SEC_S = 0, SEC_D, SEC_H0, SEC_H1, SEC_H2, SEC_O, SEC_OS, SEC_T0, SEC_T1, SEC_T2, SEC_OT, SEC_N };

struct F32Layout {
    int W;
    __host__ __device__ constexpr int mt(int s) const {
        return s == SEC_OS ? 0 : (s == SEC_O) ? 1 : W / 16;   // OS: 16-bit layout only
    }
    __host__ __device__ constexpr int kb(int s) const {
        return s == SEC_S ? 28 : s == SEC_D ? 12 : s == SEC_OT ? 4 : W / 4;
    }
    __host__ __device__ constexpr int size(int s) const { return mt(s) * kb(s) * 64; }
    __host__ __device__ constexpr int offset(int s) const {
        int o = 0;
        for (int i = 0; i < s; ++i) o += size(i);
        return o;
    }
    __host__ __device__ constexpr int total() const { return offset(SEC_N); }
};

// Canonical offsets of the five weight matrices.
__host__ __device__ constexpr int64_t w_offset(int W, int layer) {
    return layer == 0 ? 0 : (int64_t)W * kFeat + (int64_t)(layer - 1) * W * W;
}
__host__ __device__ constexpr int64_t n_params(int W) {
    return (int64_t)W * kFeat + 3LL * W * W + 3LL * W;
}

// Canonical feature index of lane group g's t-th feature of a surface (surface = true, t < 28)
// or direction (t < 12) encoding.
__host__ __device__ inline int feature_of(bool surface, int g, int t) {
    const int i = t >> 2, f = (t >> 1) & 1, sc = t & 1;
    const int input = surface ? surf_input(i) : 3 + i;
    return 16 * input + 2 * (2 * g + f) + sc;
}

// Hidden-layer neuron held at K position (kb, g) of a chained B operand.
__host__ __device__ inline int chained_neuron(int kb, int g) {
    return 16 * (kb >> 2) + 4 * g + (kb & 3);
}

// Canonical parameter index of packed FP32 element e (or -1 for zero padding).
__host__ __device__ inline int64_t f32_packed_source(int W, int e) {
    const F32Layout L{W};
    int s = 0;
    while (s + 1 < SEC_N && e >= L.offset(s + 1)) ++s;
    const int r = e - L.offset(s);
    const int KB = L.kb(s);
    const int kk = r & 3, lane = (r >> 2) & 63, rest = r >> 8;   // rest = mt * (KB/4) + kq
    const int kq = rest % (KB / 4), m = rest / (KB / 4);
    const int kb = 4 * kq + kk;
    const int row = 16 * m + (lane & 15), g = lane >> 4;
    switch (s) {
    case SEC_S: return w_offset(W, 0) + (int64_t)row * kFeat + feature_of(true, g, kb);
    case SEC_D: return w_offset(W, 0) + (int64_t)row * kFeat + feature_of(false, g, kb);
    case SEC_H0: case SEC_H1: case SEC_H2:
        return w_offset(W, 1 + (s - SEC_H0)) + (int64_t)row * W + chained_neuron(kb, g);
    case SEC_O:
        return row < 3 ? w_offset(W, 4) + (int64_t)row * W + chained_neuron(kb, g) : -1;
    case SEC_T0: case SEC_T1: case SEC_T2:
        // A = W_l^T: row = input neuron of W_l, K = output neuron of W_l (chained order)
        return w_offset(W, 1 + (s - SEC_T0)) + (int64_t)chained_neuron(kb, g) * W + row;
    case SEC_OT: {
        const int o = 4 * g + kb;   // output row held at K position (kb, g)
        return o < 3 ? w_offset(W, 4) + (int64_t)o * W + row : -1;
    }
    default: return -1;
    }
}

// The packed FP32 elements that hold canonical parameter i (the inverse of f32_packed_source):
// writes their indices to e[] and returns how many (W1: 1, W2..W5: 2, the forward and the
// transposed section).
__host__ __device__ inline int f32_packed_targets(int W, int64_t i, int (&e)[2]) {
    const F32Layout L{W};
    // element of section s holding A[row][K position (kb, g)]
    auto at = [&](int s, int row, int kb, int g) {
        const int lane = 16 * g + (row & 15);
        return L.offset(s) + (((row >> 4) * (L.kb(s) / 4) + (kb >> 2)) * 64 + lane) * 4 + (kb & 3);
    };
    // chained K position of hidden neuron n
    auto chain_kb = [](int n) { return 4 * (n >> 4) + (n & 3); };
    auto chain_g = [](int n) { return (n & 15) >> 2; };
    if (i < w_offset(W, 1)) {   // W1 [W][160]: input feature f = 16 input + 2 (2 g + fq) + sc
        const int row = (int)(i / kFeat), f = (int)(i % kFeat);
        const int input = f >> 4, k = (f & 15) >> 1, sc = f & 1;
        const bool surface = input < 3 || input > 5;
        const int pos = input < 3 ? input : input - 3;   // index in the surface or direction list
        e[0] = at(surface ? SEC_S : SEC_D, row, 4 * pos + 2 * (k & 1) + sc, k >> 1);
        return 1;
    }
    if (i < w_offset(W, 4)) {   // W2..W4 [W][W]: row r (output neuron), column c (input neuron)
        const int l = (int)((i - w_offset(W, 1)) / ((int64_t)W * W));
        const int r = (int)((i - w_offset(W, 1 + l)) / W), c = (int)((i - w_offset(W, 1 + l)) % W);
        e[0] = at(SEC_H0 + l, r, chain_kb(c), chain_g(c));
        e[1] = at(SEC_T0 + l, c, chain_kb(r), chain_g(r));
        return 2;
    }
    // W5 [3][W]: output row r sits at K position (r, 0) of the transposed section
    const int r = (int)((i - w_offset(W, 4)) / W), c = (int)((i - w_offset(W, 4)) % W);
    e[0] = at(SEC_O, r, chain_kb(c), chain_g(c));
    e[1] = at(SEC_OT, c, r, 0);
    return 2;
}

}  // namespace nirc
