// The paper's own cache input (Sec. "Neural Incident Radiance Cache", the list of encodings and
// the inference-pipeline figure): a 64-wide neural input made of
//   - 24 values of a 12-level multiresolution hash grid on the position x, 2 trainable features
//     per level (Mueller et al., Instant NGP, SIGGRAPH 2022),
//   - 25 real spherical harmonics of degree <= 4 of the direction w,
//   - 15 surface values phi: the normal (identity), the roughness as an 8-bin one-blob
//     (Mueller et al., Neural Importance Sampling, TOG 2019), the albedo (identity; the white
//     Lambertian surface has albedo 1) and one zero slot.
// Canonical input order: hash (2 l + f), SH (l^2 + l + m), normal, one-blob, albedo, zero.
// Width 64 with BF16 / FP16 MFMA operands; the grid features stay FP32 and are interpolated in
// FP32 before they become 16-bit operands.
#pragma once

#include "nirc_h16.hpp"

namespace nirc {

constexpr int kHashLevels = 12;
constexpr int kHashIn = 64;
constexpr int kHashW = 64;
constexpr int kHashMlp = kHashW * kHashIn + 3 * kHashW * kHashW + 3 * kHashW;   // 16,576

// One level of the grid: resolution N, first entry, dense flag.
struct HashLevel {
    int32_t res;
    uint32_t off;
    uint32_t dense;
    uint32_t pad;
};

struct HashGridArgs {
    HashLevel lv[kHashLevels];
    uint32_t tmask;   // T - 1 (T = 2^log2_table entries per hashed level)
    uint32_t entries;
};

// Host: levels of N_l = floor(N_0 b^l); a level is a dense (N+1)^3 table when that fits in T
// entries, otherwise T hashed entries.  Returns the total entry count (0 for a bad grid).
inline int64_t hash_grid_setup(const nirc_hash_grid &g, HashGridArgs *out) {
    if (g.log2_table < 10 || g.log2_table > 22 || g.base_res < 2 || !(g.growth >= 1.0f && g.growth <= 4.0f))
        return 0;
    const int64_t T = (int64_t)1 << g.log2_table;
    int64_t off = 0;
    double scale = 1.0;
    for (int l = 0; l < kHashLevels; ++l) {
        const double r = (double)g.base_res * scale;
        scale *= (double)g.growth;
        if (r > (double)(1 << 20)) return 0;
        const int64_t N = (int64_t)r;   // floor: r > 0
        const int64_t v = (N + 1) * (N + 1) * (N + 1);
        const bool dense = v <= T;
        if (out) out->lv[l] = HashLevel{(int32_t)N, (uint32_t)off, dense ? 1u : 0u, 0u};
        off += dense ? v : T;
    }
    if (out) {
        out->tmask = (uint32_t)(T - 1);
        out->entries = (uint32_t)off;
    }
    return off;
}

// ------------------------------------------------------------------------------------------
// Spherical harmonics: Y_lm = C_lm(z) R_m(x, y) with R_m = Re (x + iy)^m (m > 0), Im (x + iy)^|m|
// (m < 0) or 1, and C_lm the normalised associated Legendre factor (no Condon-Shortley phase)
// as a polynomial in z.  The direction is taken as unit length.
__host__ __device__ inline void sh25(float x, float y, float z, float *Y) {
    const float z2 = z * z;
    const float x2 = x * x, y2 = y * y;
    const float c2 = x2 - y2, s2 = 2.0f * x * y;           // m = 2
    const float c3 = x * (x2 - 3.0f * y2), s3 = y * (3.0f * x2 - y2);   // m = 3
    const float c4 = c2 * c2 - s2 * s2, s4 = 2.0f * c2 * s2;            // m = 4
    Y[0] = 0.28209479177387814f;
    Y[1] = 0.48860251190291992f * y;
    Y[2] = 0.48860251190291992f * z;
    Y[3] = 0.48860251190291992f * x;
    const float q21 = 1.0925484305920792f * z;
    Y[4] = 0.54627421529603959f * s2;
    Y[5] = q21 * y;
    Y[6] = 0.94617469575756008f * z2 - 0.31539156525252005f;
    Y[7] = q21 * x;
    Y[8] = 0.54627421529603959f * c2;
    const float q31 = 2.2852289973223292f * z2 - 0.45704579946446577f;
    const float q32 = 1.4453057213202773f * z;
    Y[9] = 0.59004358992664363f * s3;
    Y[10] = q32 * s2;
    Y[11] = q31 * y;
    Y[12] = z * (1.865881662950577f * z2 - 1.1195289977703462f);
    Y[13] = q31 * x;
    Y[14] = q32 * c2;
    Y[15] = 0.59004358992664363f * c3;
    const float q41 = z * (4.6833258049010249f * z2 - 2.0071396306718676f);
    const float q42 = 3.3116114351514598f * z2 - 0.47308734787877998f;
    const float q43 = 1.7701307697799307f * z;
    Y[16] = 0.62583573544917626f * s4;
    Y[17] = q43 * s3;
    Y[18] = q42 * s2;
    Y[19] = q41 * y;
    Y[20] = (3.7024941420321507f * z2 - 3.1735664074561294f) * z2 + 0.31735664074561293f;
    Y[21] = q41 * x;
    Y[22] = q42 * c2;
    Y[23] = q43 * c3;
    Y[24] = 0.62583573544917626f * c4;
}

// The 15 surface values: normal, one-blob of the roughness (8 bins, Gaussian of width 1/8 read
// at the bin centres), albedo 1, 1, 1 and a zero slot.
__host__ __device__ inline void phi_values(const float xs[7], float *ph) {
    ph[0] = xs[3];
    ph[1] = xs[4];
    ph[2] = xs[5];
    const float r8 = 8.0f * xs[6];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const float d = r8 - ((float)i + 0.5f);
        ph[3 + i] = expf(-0.5f * d * d);
    }
    ph[11] = ph[12] = ph[13] = 1.0f;
    ph[14] = 0.0f;
}

// ------------------------------------------------------------------------------------------
// 16-bit MFMA operands (16x16x32: lane (g, col) holds K positions 8g + j of a K-block).
// Surface operand, two K-blocks: block 0 carries lane group g's six grid values (levels 3g..3g+2)
// at j < 6 and phi[2g], phi[2g+1] at j = 6, 7; block 1 carries phi[8..14] in lane group 0.
// Direction operand, one K-block: SH value 8g + j (zero past 24).
__host__ __device__ inline int hash_surface_input(int kb, int g, int j) {
    if (kb == 0) return j < 6 ? 6 * g + j : 49 + 2 * g + (j - 6);
    return (g == 0 && j < 7) ? 57 + j : -1;
}
__host__ __device__ inline int hash_direction_input(int g, int j) { return 8 * g + j < 25 ? 24 + 8 * g + j : -1; }

// Packed 16-bit weights: S (W1 surface columns, 4 row tiles x 2 K-blocks), D (W1 direction
// columns, 4 x 1), then the hidden, output and transposed sections exactly as in the frequency
// model's 16-bit layout (H0..H2, O, OS, T0..T2, OT), then TS: the grid columns of W1 transposed
// as an A operand (rows = grid inputs 0..23 in 2 row tiles, K = neurons in chained order), for
// the gradient with respect to the grid values.
constexpr int kHashSecS = 0;
constexpr int kHashSecD = 4 * 2 * 512;
constexpr int kHashRest = kHashSecD + 4 * 1 * 512;
constexpr int kHashRestSize = H16Layout{64}.offset(SEC_N) - H16Layout{64}.offset(SEC_H0);
constexpr int kHashSecTS = kHashRest + kHashRestSize;
constexpr int kHashPacked = kHashSecTS + 2 * 2 * 512;
// offset of a frequency-layout section (SEC_H0 and later) inside the hash layout
__host__ __device__ constexpr int hash_sec(int s) { return kHashRest + H16Layout{64}.offset(s) - H16Layout{64}.offset(SEC_H0); }
// canonical offset of W2 (frequency model) minus that of the hash model
constexpr int64_t kHashCanonShift = (int64_t)64 * kFeat - (int64_t)64 * kHashIn;

// Canonical (hash model) parameter index of packed element e, or -1 for zero padding.
__host__ __device__ inline int64_t hash_packed_source(int e) {
    if (e < kHashSecD || (e >= kHashSecTS && e < kHashPacked) || (e >= kHashSecD && e < kHashRest)) {
        const bool ts = e >= kHashSecTS;
        const bool dir = !ts && e >= kHashSecD;
        const int r = e - (ts ? kHashSecTS : dir ? kHashSecD : kHashSecS);
        const int KB = dir ? 1 : 2;
        const int j = r & 7, lane = (r >> 3) & 63, rest = r >> 9;
        const int kb = rest % KB, m = rest / KB;
        const int row = 16 * m + (lane & 15), g = lane >> 4;
        if (ts) return row < 24 ? (int64_t)chained_neuron16(kb, g, j) * kHashIn + row : -1;
        const int in = dir ? hash_direction_input(g, j) : hash_surface_input(kb, g, j);
        return in < 0 ? -1 : (int64_t)row * kHashIn + in;
    }
    if (e >= kHashRest && e < kHashSecTS) {
        const int64_t s = h16_packed_source(64, e - kHashRest + H16Layout{64}.offset(SEC_H0));
        return s < 0 ? -1 : s - kHashCanonShift;
    }
    return -1;
}

// ------------------------------------------------------------------------------------------
// Grid lookups.

struct HashCell {
    int c[3];
    float f[3];
};

// Cell of x (clamped to the unit cube) at resolution N: lower corner and fractions.
__host__ __device__ __forceinline__ HashCell hash_cell(float x0, float x1, float x2, int N) {
    HashCell h;
    const float xs[3] = {x0, x1, x2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const float p = fminf(fmaxf(xs[d], 0.0f), 1.0f) * (float)N;
        const int ci = min((int)floorf(p), N - 1);
        h.c[d] = ci;
        h.f[d] = p - (float)ci;
    }
    return h;
}

// Entry of corner k (bit d of k: +1 along axis d) and its trilinear weight.
__host__ __device__ __forceinline__ uint32_t hash_entry(const HashLevel &lv, uint32_t tmask, const HashCell &h, int k,
                                               float &w) {
    const int v0 = h.c[0] + (k & 1), v1 = h.c[1] + ((k >> 1) & 1), v2 = h.c[2] + ((k >> 2) & 1);
    w = ((k & 1) ? h.f[0] : 1.0f - h.f[0]) * (((k >> 1) & 1) ? h.f[1] : 1.0f - h.f[1]) *
        (((k >> 2) & 1) ? h.f[2] : 1.0f - h.f[2]);
    const uint32_t n1 = (uint32_t)lv.res + 1u;
    const uint32_t dense = (uint32_t)v0 + n1 * ((uint32_t)v1 + n1 * (uint32_t)v2);
    const uint32_t hashed = ((uint32_t)v0 ^ ((uint32_t)v1 * 2654435761u) ^ ((uint32_t)v2 * 805459861u)) & tmask;
    return lv.off + (lv.dense ? dense : hashed);
}

// The 24 corner features lane group g needs at x (levels 3g..3g+2, 8 corners each): loads only,
// so that they can be issued one point group ahead of their use.  The y and z parts of the
// dense index and of the hash are formed once per level and shared by the corners.
__host__ __device__ __forceinline__ void hash_fetch24(const HashLevel *slv, uint32_t tmask, const float2 *table, float x0,
                                             float x1, float x2, int g, float2 (&t)[24]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const HashLevel lv = slv[3 * g + k];
        const HashCell h = hash_cell(x0, x1, x2, lv.res);
        const uint32_t n1 = (uint32_t)lv.res + 1u;
        const uint32_t c0 = (uint32_t)h.c[0], c1 = (uint32_t)h.c[1], c2 = (uint32_t)h.c[2];
        const uint32_t dy = n1 * (c1 + n1 * c2);                          // dense: corner (0, 0, 0)
        const uint32_t hy0 = c1 * 2654435761u, hz0 = c2 * 805459861u;     // hash: y and z parts
        const uint32_t hy1 = hy0 + 2654435761u, hz1 = hz0 + 805459861u;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const uint32_t bx = c & 1, by = (c >> 1) & 1, bz = (c >> 2) & 1;
            const uint32_t dense = c0 + bx + dy + (by ? n1 : 0u) + (bz ? n1 * n1 : 0u);
            const uint32_t hashed = ((c0 + bx) ^ (by ? hy1 : hy0) ^ (bz ? hz1 : hz0)) & tmask;
            t[8 * k + c] = table[lv.off + (lv.dense ? dense : hashed)];
        }
    }
}

// Trilinear blend of fetched corner features into lane group g's six grid values.
__host__ __device__ __forceinline__ void hash_blend6(const HashLevel *slv, float x0, float x1, float x2, int g,
                                            const float2 (&t)[24], float (&v)[6]) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const HashLevel lv = slv[3 * g + k];
        const HashCell h = hash_cell(x0, x1, x2, lv.res);
        float a = 0.0f, b = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
            const float w = ((c & 1) ? h.f[0] : 1.0f - h.f[0]) * (((c >> 1) & 1) ? h.f[1] : 1.0f - h.f[1]) *
                            (((c >> 2) & 1) ? h.f[2] : 1.0f - h.f[2]);
            a += w * t[8 * k + c].x;
            b += w * t[8 * k + c].y;
        }
        v[2 * k] = a;
        v[2 * k + 1] = b;
    }
}

// Lane group g's six grid values at x (all 24 loads issued before they are blended).
__host__ __device__ __forceinline__ void hash_values6(const HashLevel *slv, uint32_t tmask, const float2 *table, float x0,
                                             float x1, float x2, int g, float (&v)[6]) {
    float2 t[24];
    hash_fetch24(slv, tmask, table, x0, x1, x2, g, t);
    hash_blend6(slv, x0, x1, x2, g, t, v);
}

// One bin of the roughness one-blob (index i may be any value; used only where in range).
__device__ __forceinline__ float oneblob_bin(float r, float i) {
    const float d = 8.0f * r - (i + 0.5f);
    return expf(-0.5f * d * d);
}

// Surface operands from grid values already blended (v) and the point's inputs.  Lane group g
// needs phi[2g], phi[2g+1] (and group 0 also phi[8..14]): normal (phi 0..2), one-blob bins
// (phi 3..10), albedo 1 (phi 11..13), zero (phi 14); only the bins a group uses are evaluated.
template <int PREC>
__device__ __forceinline__ void hash_pack_surface(const float xs[7], int g, const float (&v)[6], u32x4 &b0,
                                                  u32x4 &b1) {
    // bins: group 0 -> 5, 6, 7 (phi 8..10); group 1 -> 0 (phi 3); group 2 -> 1, 2; group 3 -> 3, 4
    const float i0 = g == 0 ? 5.0f : g == 1 ? 0.0f : g == 2 ? 1.0f : 3.0f;
    const float e0 = oneblob_bin(xs[6], i0), e1 = oneblob_bin(xs[6], i0 + 1.0f);
    const float e2 = oneblob_bin(xs[6], 7.0f);
    const float p0 = g == 0 ? xs[3] : g == 1 ? xs[5] : e0;
    const float p1 = g == 0 ? xs[4] : g == 1 ? e0 : e1;
    b0 = u32x4{pack2<PREC>(v[0], v[1]), pack2<PREC>(v[2], v[3]), pack2<PREC>(v[4], v[5]), pack2<PREC>(p0, p1)};
    b1 = g == 0 ? u32x4{pack2<PREC>(e0, e1), pack2<PREC>(e2, 1.0f), pack2<PREC>(1.0f, 1.0f), pack2<PREC>(0.0f, 0.0f)}
                : u32x4{0u, 0u, 0u, 0u};
}

// The two surface K-blocks of lane group g for a point (grid values and phi).
template <int PREC>
__device__ __forceinline__ void hash_surface_operands(const HashLevel *slv, uint32_t tmask, const float2 *table,
                                                      const float xs[7], int g, u32x4 &b0, u32x4 &b1,
                                                      float (&v)[6], float (&ph)[15]) {
    hash_values6(slv, tmask, table, xs[0], xs[1], xs[2], g, v);
    phi_values(xs, ph);
    hash_pack_surface<PREC>(xs, g, v, b0, b1);
}

// h += W1_s e_s for one tile of 16 columns (the surface section read from global memory).
template <int PREC>
__device__ __forceinline__ void hash_layer1_surface(f32x4 (&h)[4], const uint16_t *gS, const u32x4 &b0,
                                                    const u32x4 &b1, int lane) {
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        h[mt] = mfma16<PREC>(*(const u32x4 *)(gS + ((mt * 2 + 0) * 64 + lane) * 8), b0, h[mt]);
        h[mt] = mfma16<PREC>(*(const u32x4 *)(gS + ((mt * 2 + 1) * 64 + lane) * 8), b1, h[mt]);
    }
}

// Eight consecutive values from Y[B] as one operand (constant indices only).
template <int PREC, int B>
__device__ __forceinline__ u32x4 pack8(const float *Y) {
    return u32x4{pack2<PREC>(Y[B], Y[B + 1]), pack2<PREC>(Y[B + 2], Y[B + 3]), pack2<PREC>(Y[B + 4], Y[B + 5]),
                 pack2<PREC>(Y[B + 6], Y[B + 7])};
}

// Direction operand of lane group g from the 25 SH values: the four candidates are packed and
// one is selected by value (selecting array elements by g would put Y in scratch memory).
template <int PREC>
__device__ __forceinline__ u32x4 sh_operand_of(const float *Y, int g) {
    const u32x4 o0 = pack8<PREC, 0>(Y), o1 = pack8<PREC, 8>(Y), o2 = pack8<PREC, 16>(Y);
    const u32x4 o3 = u32x4{pack2<PREC>(Y[24], 0.0f), 0u, 0u, 0u};
    return g == 0 ? o0 : g == 1 ? o1 : g == 2 ? o2 : o3;
}

template <int PREC>
__device__ __forceinline__ u32x4 sh_operand(float dx, float dy, float dz, int g) {
    float Y[25];
    sh25(dx, dy, dz, Y);
    return sh_operand_of<PREC>(Y, g);
}

// All four lane groups' direction operands of one query, written with stride `stride`.
template <int PREC>
__device__ __forceinline__ void sh_features16(float dx, float dy, float dz, u32x4 *fa, int stride) {
    float Y[25];
    sh25(dx, dy, dz, Y);
    fa[0] = pack8<PREC, 0>(Y);
    fa[stride] = pack8<PREC, 8>(Y);
    fa[2 * stride] = pack8<PREC, 16>(Y);
    fa[3 * stride] = u32x4{pack2<PREC>(Y[24], 0.0f), 0u, 0u, 0u};
}

// Stages the grid levels in LDS (constant indices only, so the argument array is never indexed
// by lane).
__device__ __forceinline__ void stage_levels(HashLevel *slv, const HashGridArgs &grid) {
#pragma unroll
    for (int l = 0; l < kHashLevels; ++l)
        if ((int)threadIdx.x == l) slv[l] = grid.lv[l];
}


// ------------------------------------------------------------------------------------------
// FP32 chain (16x16x4 MFMA: lane group g holds K index g of each K-step), inference only.
// Packed FP32 weights: S (W1 surface columns: 4 row tiles x 12 K-steps), D (W1 direction
// columns: 4 x 8), then H0..H2 and O exactly as in the frequency model's FP32 layout.  K-step k
// of lane group g carries canonical input
//   S: k < 6: grid value 6g + k (levels 3g..3g+2); 6 <= k < 10: surface value phi[4(k-6) + g]
//      (none past phi 14); k = 10, 11: zero;
//   D: k < 7: spherical harmonic 4k + g (none past 24); k = 7: zero.
constexpr int kHash32S = 4 * 12 * 64;
constexpr int kHash32D = 4 * 8 * 64;
constexpr int kHash32Rest = F32Layout{64}.offset(SEC_T0) - F32Layout{64}.offset(SEC_H0);   // H0..H2, O
// training sections after the inference ones: T0..T2 and OT as in the frequency model's FP32
// layout, then TS32 (W1's grid columns transposed: rows = grid inputs in 2 row tiles, K = neurons
// in the FP32 chained order, 16 K-steps)
constexpr int kHash32T = F32Layout{64}.offset(SEC_N) - F32Layout{64}.offset(SEC_T0);
constexpr int kHash32TS = kHash32S + kHash32D + kHash32Rest + kHash32T;
constexpr int kHash32Packed = kHash32TS + 2 * 16 * 64;
// offset of a frequency-layout FP32 section (SEC_H0 and later) inside the hash FP32 layout
__host__ __device__ constexpr int hash_sec32(int s) {
    return kHash32S + kHash32D + F32Layout{64}.offset(s) - F32Layout{64}.offset(SEC_H0);
}

__host__ __device__ inline int64_t hash_packed_source32(int e) {
    if (e < kHash32S + kHash32D) {
        const bool dir = e >= kHash32S;
        const int r = e - (dir ? kHash32S : 0);
        const int NQ = dir ? 2 : 3;   // K-quads
        const int kk = r & 3, lane = (r >> 2) & 63, rest = r >> 8;
        const int kq = rest % NQ, m = rest / NQ;
        const int k = 4 * kq + kk, row = 16 * m + (lane & 15), g = lane >> 4;
        int in = -1;
        if (dir) {
            if (k < 7 && 4 * k + g < 25) in = 24 + 4 * k + g;
        } else if (k < 6) {
            in = 6 * g + k;
        } else if (k < 10 && 4 * (k - 6) + g < 15) {
            in = 49 + 4 * (k - 6) + g;
        }
        return in < 0 ? -1 : (int64_t)row * kHashIn + in;
    }
    if (e < kHash32TS) {
        const int64_t s = f32_packed_source(64, e - kHash32S - kHash32D + F32Layout{64}.offset(SEC_H0));
        return s < 0 ? -1 : s - kHashCanonShift;
    }
    if (e < kHash32Packed) {
        const int r = e - kHash32TS;
        const int kk = r & 3, lane = (r >> 2) & 63, rest = r >> 8;   // rest = mt * 4 + kq
        const int kq = rest % 4, m = rest / 4;
        const int kb = 4 * kq + kk, row = 16 * m + (lane & 15), g = lane >> 4;
        return row < 24 ? (int64_t)chained_neuron(kb, g) * kHashIn + row : -1;
    }
    return -1;
}

// phi[4j + g], j = 0..3, for lane group g (normal, one-blob bins, albedo 1, zero slot, pad).
// (The surface values come in as scalars so that the normal's selection stays a select of values.)
__device__ __forceinline__ void hash_phi4(float nx, float ny, float nz, float rough, int g, float (&ph)[4]) {
    // bins needed: g < 3: g + 1 and g + 5; g = 3: 4 and 0
    const float ia = g < 3 ? (float)(g + 1) : 4.0f, ib = g < 3 ? (float)(g + 5) : 0.0f;
    const float ea = oneblob_bin(rough, ia), eb = oneblob_bin(rough, ib);
    const float nrm = g == 0 ? nx : g == 1 ? ny : nz;
    ph[0] = g < 3 ? nrm : eb;                  // phi[g]: normal, or bin 0
    ph[1] = ea;                                // phi[4 + g]: bins 1..4
    ph[2] = g < 3 ? eb : 1.0f;                 // phi[8 + g]: bins 5..7, albedo
    ph[3] = g < 2 ? 1.0f : 0.0f;               // phi[12 + g]: albedo, albedo, zero slot, pad
}

// h += W1_s e_s for one tile of 16 points (FP32; surface section read from global memory).
__device__ __forceinline__ void hash_layer1_surface_f32(f32x4 (&h)[4], const float *gS, const float (&v)[6],
                                                        const float (&ph)[4], int lane) {
    const float b[12] = {v[0], v[1], v[2], v[3], v[4], v[5], ph[0], ph[1], ph[2], ph[3], 0.0f, 0.0f};
#pragma unroll
    for (int kq = 0; kq < 3; ++kq) {
        f32x4 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = *(const f32x4 *)(gS + ((mt * 3 + kq) * 64 + lane) * 4);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) h[mt] = mfma4(a[mt][kk], b[4 * kq + kk], h[mt]);
    }
}

// The 8 direction K values of lane group g: SH 4k + g (constant indices only, so the SH values
// stay in registers).
__device__ __forceinline__ void hash_dir_values_f32(float dx, float dy, float dz, int g, float (&s)[8]) {
    float Y[25];
    sh25(dx, dy, dz, Y);
    s[0] = g == 0 ? Y[0] : g == 1 ? Y[1] : g == 2 ? Y[2] : Y[3];
    s[1] = g == 0 ? Y[4] : g == 1 ? Y[5] : g == 2 ? Y[6] : Y[7];
    s[2] = g == 0 ? Y[8] : g == 1 ? Y[9] : g == 2 ? Y[10] : Y[11];
    s[3] = g == 0 ? Y[12] : g == 1 ? Y[13] : g == 2 ? Y[14] : Y[15];
    s[4] = g == 0 ? Y[16] : g == 1 ? Y[17] : g == 2 ? Y[18] : Y[19];
    s[5] = g == 0 ? Y[20] : g == 1 ? Y[21] : g == 2 ? Y[22] : Y[23];
    s[6] = g == 0 ? Y[24] : 0.0f;
    s[7] = 0.0f;
}

// h[tt] += W1_w e_w(direction of tile tt) for T tiles (FP32).
template <int T>
__device__ __forceinline__ void hash_layer1_direction_f32(f32x4 (&h)[T][4], const float *sD, const float *dx,
                                                          const float *dy, const float *dz, int lane, int g) {
    float b[T][8];
#pragma unroll
    for (int tt = 0; tt < T; ++tt) hash_dir_values_f32(dx[tt], dy[tt], dz[tt], g, b[tt]);
#pragma unroll
    for (int kq = 0; kq < 2; ++kq) {
        f32x4 a[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) a[mt] = *(const f32x4 *)(sD + ((mt * 2 + kq) * 64 + lane) * 4);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk)
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma4(a[mt][kk], b[tt][4 * kq + kk], h[tt][mt]);
    }
}

// Launchers (host).
hipError_t launch_hash_pack16(uint16_t *packed, const float *master, int prec, hipStream_t s, int64_t *step = nullptr,
                              uint32_t *flags = nullptr, uint32_t *bad = nullptr);
hipError_t launch_hash_pack32(float *packed, const float *master, hipStream_t s, int64_t *step = nullptr,
                              uint32_t *flags = nullptr, uint32_t *bad = nullptr);
// Grid-entry gradients are summed in fixed point (integer adds are associative, so the sum does
// not depend on the order the atomics land in): each contribution v (already multiplied by the
// loss scale, so of order one) is added as round(v 2^kGridFix) to a 64-bit accumulator; a
// non-finite or out-of-range contribution raises *nonfinite instead.
constexpr int kGridFix = 36;
struct GridAcc {
    unsigned long long *acc;   // [2 entries] 64-bit two's-complement sums
    uint32_t *nonfinite;       // raised (1) when a contribution cannot be represented
};

__device__ __forceinline__ void grid_acc_add(const GridAcc &g, size_t i, float v) {
    if (v == 0.0f) return;
    const float x = v * 0x1p36f;
    if (!(fabsf(x) < 0x1p62f)) {   // also catches NaN
        atomicOr(g.nonfinite, 1u);
        return;
    }
    atomicAdd(g.acc + i, (unsigned long long)llrintf(x));
}

// grad[i] = (acc[i] 2^-kGridFix) * scale for i < n, or NaN everywhere when *nonfinite; raises
// `bad` on a non-finite result.
hipError_t launch_grid_acc_finish(const GridAcc &g, float *grad, int64_t n, float scale, uint32_t *bad,
                                  hipStream_t s);

hipError_t launch_hash_grad32(const Points &pts, const Queries &q, const float *packed, const float *table,
                              const HashGridArgs &grid, TrainArgs a, float *partials, float *loss_partials,
                              GridAcc gacc, int nblocks, hipStream_t s);
hipError_t launch_hash_infer32(const Points &pts, const Queries &q, const float *packed, const float *table,
                               const HashGridArgs &grid, float *rgb, hipStream_t s);
hipError_t launch_hash_tlmc32(const Points &pts, const nirc_lobes &lobes, const float *packed, const float *table,
                              const HashGridArgs &grid, int n_cache, uint64_t seed, uint64_t frame, const float *rrad,
                              float *out_tl, float *out_c, float *out_r, hipStream_t s);
hipError_t launch_hash_infer(int prec, const Points &pts, const Queries &q, const uint16_t *packed, const float *table,
                             const HashGridArgs &grid, float *rgb, hipStream_t s);
hipError_t launch_hash_tlmc(int prec, const Points &pts, const nirc_lobes &lobes, const uint16_t *packed,
                            const float *table, const HashGridArgs &grid, int n_cache, uint64_t seed, uint64_t frame,
                            const float *rrad, float *out_tl, float *out_c, float *out_r, hipStream_t s);
// Gradient partials of the MLP ([nblocks][16,576]) and the grid-entry gradient, accumulated with
// atomics into gtab ([entries][2], zeroed by the caller); both carry the loss scale of `a`.
hipError_t launch_hash_grad(int prec, const Points &pts, const Queries &q, const uint16_t *packed, const float *table,
                            const HashGridArgs &grid, TrainArgs a, float *partials, float *loss_partials,
                            GridAcc gacc, int nblocks, hipStream_t s);

}  // namespace nirc
