// 16-bit (BF16 / FP16) MLP chain on v_mfma_f32_16x16x32_{bf16,f16}: FP32 accumulation, 16-bit
// operands, weights packed so that consecutive layers chain through registers.
#pragma once

#include "nirc_kernels.hpp"

namespace nirc {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));   // 8 16-bit values (one operand)
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef short i16x2 __attribute__((ext_vector_type(2)));

// ------------------------------------------------------------------------------------------
// Layout.  MFMA 16x16x32: lane l holds A[row l%16][k 8(l/16) + j] and B[k 8(l/16) + j][col l%16],
// j = 0..7; the result gives lane l rows 4(l/16) + i of column l%16 (as for 16x16x4).  K-block b
// of a chained layer is built from result row tiles 2b (positions j < 4) and 2b + 1 (j >= 4):
//   K position 32 b + 8 g + j  <->  neuron 32 b + 16 (j / 4) + 4 g + j % 4.
// Input features: lane group g holds the same 28 surface / 12 direction features as in the FP32
// layout (frequencies 2g, 2g+1 of every input); feature t goes to K-block t / 8, position t % 8,
// and positions past the last feature are zero.
// Sections (MT row tiles x KB K-blocks x 64 lanes x 8 values, stored [mt][kb][lane][8]):
//   S  W1 surface    MT = W/16, KB = 4     D  W1 direction  MT = W/16, KB = 2
//   H0..H2 W2..W4    MT = W/16, KB = W/32  O  W5           MT = 1,    KB = W/32
//   OS W5^T as a B operand, 4 column-shifted copies (MT = 4 copies, KB = W/32): copy t holds
//      W5 row c in column 3t + c, so that Y = H W5^T of 4 tiles accumulates into one result
//   T0..T2 W2^T..W4^T MT = W/16, KB = W/32 OT W5^T          MT = W/16, KB = 1
struct H16Layout {
    int W;
    __host__ __device__ constexpr int mt(int s) const { return s == SEC_O ? 1 : s == SEC_OS ? 4 : W / 16; }
    __host__ __device__ constexpr int kb(int s) const {
        return s == SEC_S ? 4 : s == SEC_D ? 2 : s == SEC_OT ? 1 : W / 32;
    }
    __host__ __device__ constexpr int size(int s) const { return mt(s) * kb(s) * 512; }
    __host__ __device__ constexpr int offset(int s) const {
        int o = 0;
        for (int i = 0; i < s; ++i) o += size(i);
        return o;
    }
    __host__ __device__ constexpr int total() const { return offset(SEC_N); }
};

__host__ __device__ inline int chained_neuron16(int kb, int g, int j) {
    return 32 * kb + 16 * (j >> 2) + 4 * g + (j & 3);
}

// Canonical parameter index of packed 16-bit element e (or -1 for zero padding).
__host__ __device__ inline int64_t h16_packed_source(int W, int e) {
    const H16Layout L{W};
    int s = 0;
    while (s + 1 < SEC_N && e >= L.offset(s + 1)) ++s;
    const int r = e - L.offset(s);
    const int KB = L.kb(s);
    const int j = r & 7, lane = (r >> 3) & 63, rest = r >> 9;
    const int kb = rest % KB, m = rest / KB;
    const int row = 16 * m + (lane & 15), g = lane >> 4;
    const int t = 8 * kb + j;
    switch (s) {
    case SEC_S: return t < 28 ? w_offset(W, 0) + (int64_t)row * kFeat + feature_of(true, g, t) : -1;
    case SEC_D: return t < 12 ? w_offset(W, 0) + (int64_t)row * kFeat + feature_of(false, g, t) : -1;
    case SEC_H0: case SEC_H1: case SEC_H2:
        return w_offset(W, 1 + (s - SEC_H0)) + (int64_t)row * W + chained_neuron16(kb, g, j);
    case SEC_O:
        return row < 3 ? w_offset(W, 4) + (int64_t)row * W + chained_neuron16(kb, g, j) : -1;
    case SEC_OS: {
        // B operand: lane l holds B[k = 8g + j][column l%16]; copy m puts W5 row c at column 3m + c
        const int c = (lane & 15) - 3 * m;
        return (c >= 0 && c < 3) ? w_offset(W, 4) + (int64_t)c * W + chained_neuron16(kb, g, j) : -1;
    }
    case SEC_T0: case SEC_T1: case SEC_T2:
        return w_offset(W, 1 + (s - SEC_T0)) + (int64_t)chained_neuron16(kb, g, j) * W + row;
    case SEC_OT: {
        const int o = 4 * g + j;   // output row at (g, j < 4); j >= 4 would be a second tile
        return (j < 4 && o < 3) ? w_offset(W, 4) + (int64_t)o * W + row : -1;
    }
    default: return -1;
    }
}

// The packed 16-bit elements that hold canonical parameter i (the inverse of h16_packed_source):
// writes their indices to e[] and the scale each stores (h16_packed_scale) to sc[]; returns how
// many (W1: 1, W2..W4: 2 (forward and transposed sections), W5: 6 (O, four OS copies, OT)).
__host__ __device__ inline int h16_packed_targets(int W, int64_t i, int (&e)[6], float (&sc)[6]) {
    const H16Layout L{W};
    const int KB = W / 32;
    // chained position of hidden neuron n: K-block, lane group and slot
    auto chain_pos = [](int n, int &kb, int &g, int &j) {
        kb = n >> 5;
        const int r = n & 31;
        g = (r & 15) >> 2;
        j = 4 * (r >> 4) + (r & 3);
    };
    if (i < w_offset(W, 1)) {   // W1 [W][160]
        const int row = (int)(i / kFeat), f = (int)(i % kFeat);
        const int input = f >> 4, k = (f & 15) >> 1, s_c = f & 1;
        const int g = k >> 1, fq = k & 1;
        const bool surface = input < 3 || input > 5;
        const int pos = surface ? (input < 3 ? input : input - 3) : input - 3;   // index in its list
        const int t = 4 * pos + 2 * fq + s_c;
        const int sec = surface ? SEC_S : SEC_D, kbs = surface ? 4 : 2;
        const int lane = 16 * g + (row & 15), m = row >> 4;
        e[0] = L.offset(sec) + ((m * kbs + (t >> 3)) * 64 + lane) * 8 + (t & 7);
        sc[0] = s_c ? 0.5f : 1.0f;
        return 1;
    }
    if (i < w_offset(W, 4)) {   // W2..W4 [W][W]: forward section and transposed section
        const int l = (int)((i - w_offset(W, 1)) / ((int64_t)W * W));
        const int r = (int)((i - w_offset(W, 1 + l)) / W), c = (int)((i - w_offset(W, 1 + l)) % W);
        int kb, g, j;
        chain_pos(c, kb, g, j);   // forward: row r, K position of neuron c
        e[0] = L.offset(SEC_H0 + l) + (((r >> 4) * KB + kb) * 64 + 16 * g + (r & 15)) * 8 + j;
        chain_pos(r, kb, g, j);   // transposed: row c, K position of neuron r
        e[1] = L.offset(SEC_T0 + l) + (((c >> 4) * KB + kb) * 64 + 16 * g + (c & 15)) * 8 + j;
        sc[0] = sc[1] = 1.0f;
        return 2;
    }
    // W5 [3][W]
    const int r = (int)((i - w_offset(W, 4)) / W), c = (int)((i - w_offset(W, 4)) % W);
    int kb, g, j;
    chain_pos(c, kb, g, j);
    e[0] = L.offset(SEC_O) + (kb * 64 + 16 * g + r) * 8 + j;
    for (int m = 0; m < 4; ++m) e[1 + m] = L.offset(SEC_OS) + ((m * KB + kb) * 64 + 16 * g + 3 * m + r) * 8 + j;
    e[5] = L.offset(SEC_OT) + ((c >> 4) * 64 + (c & 15)) * 8 + r;
    for (int k = 0; k < 6; ++k) sc[k] = 1.0f;
    return 6;
}

// Scale applied to packed element e: the 16-bit input features carry 2 cos instead of cos
// (angle doubling is then one multiply and one FMA per step), so the weights of the cosine
// features (odd positions of the S and D sections) are stored halved.  Halving is exact in
// both 16-bit formats (barring FP16 subnormals).
__host__ __device__ inline float h16_packed_scale(int W, int e) {
    const H16Layout L{W};
    const bool feat = (e >= L.offset(SEC_S) && e < L.offset(SEC_D) + L.size(SEC_D));
    return (feat && (e & 1)) ? 0.5f : 1.0f;
}

// ------------------------------------------------------------------------------------------
// Precision traits: PREC = NIRC_BF16 or NIRC_FP16.

template <int PREC>
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    const f32x2 v = {a, b};
    if constexpr (PREC == NIRC_BF16) return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf16x2));
    else return __builtin_bit_cast(uint32_t, __builtin_convertvector(v, f16x2));
}

// ReLU on two packed 16-bit values: both formats keep the sign in the top bit, so a signed
// 16-bit max with 0 clears negatives (and -0).
__device__ __forceinline__ uint32_t relu2(uint32_t x) {
    i16x2 v = __builtin_bit_cast(i16x2, x);
    const i16x2 z = {0, 0};
    v = v > z ? v : z;
    return __builtin_bit_cast(uint32_t, v);
}

template <int PREC>
__device__ __forceinline__ f32x4 mfma16(u32x4 a, u32x4 b, f32x4 c) {
    if constexpr (PREC == NIRC_BF16)
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    else
        return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8, a), __builtin_bit_cast(f16x8, b), c,
                                                      0, 0, 0);
}

// Features in the 16-bit chain are pairs (sin a, 2 cos a): with u = 2 cos a, doubling the angle
// is sin 2a = u sin a and 2 cos 2a = u^2 - 2.
// sin(pi 2^k v) and 2 cos(pi 2^k v) for k = 2g and 2g + 1: the hardware sine/cosine (argument in
// revolutions) at the lower frequency, then one doubling.  Accurate to ~1e-6, far below 16-bit
// rounding.
__device__ __forceinline__ void enc_pair2_fast(float v, int g, float &s0, float &u0, float &s1, float &u1) {
    const float rev = ldexpf(v, 2 * g - 1);   // 2^(2g) pi v in revolutions
    s0 = __builtin_amdgcn_sinf(rev);
    u0 = 2.0f * __builtin_amdgcn_cosf(rev);
    s1 = s0 * u0;
    u1 = u0 * u0 - 2.0f;
}

// All eight frequencies of one coordinate as packed 16-bit (sin, 2 cos) pairs, by seven angle
// doublings from k = 0 (each doubling at most doubles the FP32 error: ~1e-5 at k = 7).
template <int PREC>
__device__ __forceinline__ void chain8(float v, uint32_t (&p)[8]) {
    float s = __builtin_amdgcn_sinf(0.5f * v);   // sin(pi v); argument in revolutions
    float u = 2.0f * __builtin_amdgcn_cosf(0.5f * v);
    p[0] = pack2<PREC>(s, u);
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        const float s2 = s * u;
        u = u * u - 2.0f;
        s = s2;
        p[k] = pack2<PREC>(s, u);
    }
}

// Direction features of one query for all four lane groups, in the order of the D section's
// B operands: fa[g] = x(2g), x(2g+1), y(2g), y(2g+1) and fb[g] = z(2g), z(2g+1) (each a packed
// (sin, 2 cos) pair).  `stride` is the distance between consecutive lane groups' entries.
template <int PREC>
__device__ __forceinline__ void dir_features16(float dx, float dy, float dz, u32x4 *fa, uint2 *fb, int stride) {
    uint32_t px[8], py[8], pz[8];
    chain8<PREC>(dx, px);
    chain8<PREC>(dy, py);
    chain8<PREC>(dz, pz);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
        fa[g * stride] = u32x4{px[2 * g], px[2 * g + 1], py[2 * g], py[2 * g + 1]};
        fb[g * stride] = make_uint2(pz[2 * g], pz[2 * g + 1]);
    }
}

// B operand (two K-blocks of the chain) from two result tiles, with ReLU.
template <int PREC>
__device__ __forceinline__ u32x4 chain_operand(const f32x4 &lo, const f32x4 &hi) {
    return u32x4{relu2(pack2<PREC>(lo[0], lo[1])), relu2(pack2<PREC>(lo[2], lo[3])),
                 relu2(pack2<PREC>(hi[0], hi[1])), relu2(pack2<PREC>(hi[2], hi[3]))};
}

// h += W1_s e_s for one tile of 16 columns (surface features in B layout, 4 K-blocks).
template <int W, int PREC>
__device__ __forceinline__ void layer1_surface16(f32x4 (&h)[W / 16], const uint16_t *gS, const float xs[7],
                                                 int lane, int g) {
    constexpr int MT = W / 16;
    float f[32];
#pragma unroll
    for (int i = 0; i < 7; ++i) enc_pair2_fast(xs[i], g, f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
    f[28] = f[29] = f[30] = f[31] = 0.0f;
#pragma unroll
    for (int kb = 0; kb < 4; ++kb) {
        const u32x4 b = {pack2<PREC>(f[8 * kb], f[8 * kb + 1]), pack2<PREC>(f[8 * kb + 2], f[8 * kb + 3]),
                         pack2<PREC>(f[8 * kb + 4], f[8 * kb + 5]), pack2<PREC>(f[8 * kb + 6], f[8 * kb + 7])};
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            const u32x4 a = *(const u32x4 *)(gS + ((mt * 4 + kb) * 64 + lane) * 8);
            h[mt] = mfma16<PREC>(a, b, h[mt]);
        }
    }
}

// Direction features of one tile as two B operands.
template <int PREC>
__device__ __forceinline__ void direction_operands(float dx, float dy, float dz, int g, u32x4 &b0, u32x4 &b1) {
    float f[12];
    enc_pair2_fast(dx, g, f[0], f[1], f[2], f[3]);
    enc_pair2_fast(dy, g, f[4], f[5], f[6], f[7]);
    enc_pair2_fast(dz, g, f[8], f[9], f[10], f[11]);
    b0 = u32x4{pack2<PREC>(f[0], f[1]), pack2<PREC>(f[2], f[3]), pack2<PREC>(f[4], f[5]), pack2<PREC>(f[6], f[7])};
    b1 = u32x4{pack2<PREC>(f[8], f[9]), pack2<PREC>(f[10], f[11]), 0u, 0u};
}

// Layer 1 (direction part, accumulating onto h) + ReLU, then layers 2..4, for T tiles; leaves
// the hidden activations of layer 4 as chained B operands hb[tt][kb].  Each layer's weight
// fragments are fetched from LDS while the previous layer's MFMAs drain and its epilogue runs
// (software prefetch), so LDS latency does not sit between the layers.  `next` receives the
// output layer's fragments (4 shifted copies x KB) for output16_packed.
// The direction-layer fragments (`dfrag`, [kb][mt], from load_dir_fragments) stay in registers
// across passes.
// DKB: K-blocks of the direction section (2 for the frequency input, 1 for spherical harmonics).
template <int W, int DKB = 2>
__device__ __forceinline__ void load_dir_fragments(u32x4 (&dfrag)[W / 8], const uint16_t *sD, int lane) {
    constexpr int MT = W / 16;
#pragma unroll
    for (int kb = 0; kb < DKB; ++kb)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
            dfrag[kb * MT + mt] = *(const u32x4 *)(sD + ((mt * DKB + kb) * 64 + lane) * 8);
}

template <int W, int PREC, int T, int DKB = 2>
__device__ __forceinline__ void mlp16(f32x4 (&h)[T][W / 16], u32x4 (&hb)[T][W / 32], const u32x4 (&bd)[T][2],
                                      const u32x4 (&dfrag)[W / 8], const uint16_t *sH, const uint16_t *sOS, int lane,
                                      u32x4 (&aout)[4 * (W / 32)]) {
    constexpr int MT = W / 16, KB = W / 32;
    static_assert(KB == 2, "fragment buffer sized for KB = 2");
    u32x4 a[MT * 2];   // fragments of the hidden layer being computed: [kb][mt]
#pragma unroll
    for (int layer = 0; layer < 4; ++layer) {
        __builtin_amdgcn_sched_barrier(0);
        const u32x4(&bin)[T][2] = layer == 0 ? bd : hb;
        const u32x4(&af)[MT * 2] = layer == 0 ? dfrag : a;
        if (layer > 0) {
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[tt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        // the wave's MFMA run at raised issue priority: the SIMD's other wave fills the gaps
        // with its VALU work (measured: 1.5 % shorter estimates)
        __builtin_amdgcn_s_setprio(1);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kb = 0; kb < (layer == 0 ? DKB : 2); ++kb)
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma16<PREC>(af[kb * MT + mt], bin[tt][kb], h[tt][mt]);
        __builtin_amdgcn_sched_barrier(0);
        __builtin_amdgcn_s_setprio(0);
        // prefetch the next layer's fragments (hidden layer `layer`, or the output copies)
        if (layer < 3) {
            const uint16_t *sec = sH + layer * (MT * KB * 512);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a[kb * MT + mt] = *(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8);
        } else {
#pragma unroll
            for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4)
                    aout[kb * 4 + t4] = *(const u32x4 *)(sOS + ((t4 * KB + kb) * 64 + lane) * 8);
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) hb[tt][kb] = chain_operand<PREC>(h[tt][2 * kb], h[tt][2 * kb + 1]);
    }
}

// The same chain for widths above 64, whose weights stay in global memory: fragments are loaded
// one K-block (MT fragments) at a time, and only the T shifted output copies the pass needs.
template <int W, int PREC, int T>
__device__ __forceinline__ void mlp16_wide(f32x4 (&h)[T][W / 16], u32x4 (&hb)[T][W / 32], const u32x4 (&bd)[T][2],
                                           const uint16_t *sD, const uint16_t *sH, const uint16_t *sOS, int lane,
                                           u32x4 (&aout)[4 * (W / 32)]) {
    constexpr int MT = W / 16, KB = W / 32;
#pragma unroll
    for (int layer = 0; layer < 4; ++layer) {
        __builtin_amdgcn_sched_barrier(0);
        if (layer > 0) {
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[tt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        if (layer == 0) {
#pragma unroll
            for (int kb = 0; kb < 2; ++kb) {
                u32x4 a[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a[mt] = *(const u32x4 *)(sD + ((mt * 2 + kb) * 64 + lane) * 8);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma16<PREC>(a[mt], bd[tt][kb], h[tt][mt]);
            }
        } else {
            const uint16_t *sec = sH + (layer - 1) * (MT * KB * 512);
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) {
                u32x4 a[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a[mt] = *(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma16<PREC>(a[mt], hb[tt][kb], h[tt][mt]);
            }
        }
#pragma unroll
        for (int tt = 0; tt < T; ++tt)
#pragma unroll
            for (int kb = 0; kb < KB; ++kb) hb[tt][kb] = chain_operand<PREC>(h[tt][2 * kb], h[tt][2 * kb + 1]);
    }
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int t4 = 0; t4 < T; ++t4) aout[kb * 4 + t4] = *(const u32x4 *)(sOS + ((t4 * KB + kb) * 64 + lane) * 8);
}

// The chain for widths above 64 with the hidden layers' fragments in LDS (sH), the direction
// layer's fragments (dfrag, [kb][mt]) loaded from global memory by the caller before it builds
// the pass's direction operands, and the output copies in global memory: every hidden K-block's
// fragments are loaded one K-block ahead
// (double buffer) so that LDS latency sits under the previous K-block's MFMAs, and the output
// copies are requested when the last hidden layer starts.
template <int W, int PREC, int T>
__device__ __forceinline__ void mlp16_hl(f32x4 (&h)[T][W / 16], u32x4 (&hb)[T][W / 32], const u32x4 (&bd)[T][2],
                                         const u32x4 (&dfrag)[W / 8], const uint16_t *sH, const uint16_t *gOS,
                                         int lane, u32x4 (&aout)[4 * (W / 32)]) {
    constexpr int MT = W / 16, KB = W / 32, SEC = MT * KB * 512, NI = 3 * KB;
    u32x4 a[2][MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) a[0][mt] = *(const u32x4 *)(sH + ((mt * KB) * 64 + lane) * 8);
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma16<PREC>(dfrag[kb * MT + mt], bd[tt][kb], h[tt][mt]);
#pragma unroll
    for (int tt = 0; tt < T; ++tt)
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) hb[tt][kb] = chain_operand<PREC>(h[tt][2 * kb], h[tt][2 * kb + 1]);
#pragma unroll
    for (int i = 0; i < NI; ++i) {
        const int kb = i % KB;
        if (kb == 0) {
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[tt][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
        if (i == NI - KB) {
#pragma unroll
            for (int k = 0; k < KB; ++k)
#pragma unroll
                for (int t4 = 0; t4 < T; ++t4) aout[k * 4 + t4] = *(const u32x4 *)(gOS + ((t4 * KB + k) * 64 + lane) * 8);
        }
        if (i + 1 < NI) {
            const int l1 = (i + 1) / KB, kb1 = (i + 1) % KB;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
                a[(i + 1) & 1][mt] = *(const u32x4 *)(sH + l1 * SEC + ((mt * KB + kb1) * 64 + lane) * 8);
        }
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int tt = 0; tt < T; ++tt) h[tt][mt] = mfma16<PREC>(a[i & 1][mt], hb[tt][kb], h[tt][mt]);
        if (kb == KB - 1) {
#pragma unroll
            for (int tt = 0; tt < T; ++tt)
#pragma unroll
                for (int k = 0; k < KB; ++k) hb[tt][k] = chain_operand<PREC>(h[tt][2 * k], h[tt][2 * k + 1]);
        }
    }
}

// Output layer for T <= 4 tiles into ONE accumulator: the chained activations hb[tt] (B layout:
// lane l holds neuron positions 8g + j of query l%16) are exactly an A operand of the transposed
// product Y = H W5^T (A[query l%16][k 8g + j]), and shifted copy tt of W5^T sends tile tt to
// columns 3tt..3tt+2.  Lane (g, col) ends with z of queries 4g + i (i = 0..3) of tile col / 3,
// channel col % 3 (columns >= 3T are zero).
template <int W, int PREC, int T>
__device__ __forceinline__ f32x4 output16_packed(const u32x4 (&hb)[T][W / 32], const u32x4 (&aout)[4 * (W / 32)]) {
    constexpr int KB = W / 32;
    __builtin_amdgcn_sched_barrier(0);
    f32x4 y = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int tt = 0; tt < T; ++tt) y = mfma16<PREC>(hb[tt][kb], aout[kb * 4 + tt], y);
    return y;
}

}  // namespace nirc
