// Training kernels: fused forward + relative-L2 loss + backward to per-workgroup weight-gradient
// partials, a fixed-order reduction, and Adam with a refresh of the packed weights.
#include "nirc_hash.hpp"

namespace nirc {

namespace {

constexpr int kTrainWaves = 4;
constexpr int kChunk = 16 * kTrainWaves;   // samples staged per round
constexpr int kStride = kChunk + 4;        // LDS row stride (floats): conflict-free 16 B reads

template <int W>
struct GradLds {
    static constexpr int kH = 4 * W * kStride;     // h1..h4   [layer][neuron][sample]
    static constexpr int kD = 4 * W * kStride;     // delta1..delta4
    static constexpr int kD5 = 4 * kStride;        // output-layer delta, rows 0..3
    static constexpr int kX = kChunk * kInputs;    // raw inputs [sample][10]
    static constexpr int kLoss = kTrainWaves;
    static constexpr int kTotal = kH + kD + kD5 + kX + kLoss;
};

// Output-pre-activation gradient and loss term of one channel.
// rel: the relative loss (denominator y^2 + eps held constant), else den = 1; fr: the F_r shift of
// the residual-variance loss (0 otherwise)
// sig: sigmoid outputs (dy/dz = y (1 - y)) instead of exp (dy/dz = y)
__device__ inline float out_grad(float z, float t, float dr, bool use_loss, float eps, float k, bool rel,
                                 float fr, bool sig, float &loss_term) {
    const float y = sig ? logistic(z) : expf(z);
    const float dydz = sig ? y * (1.0f - y) : y;
    if (use_loss) {
        const float d = (y - t) + fr, den = rel ? y * y + eps : 1.0f;
        loss_term = d * d / den;
        return k * d / den * dydz;   // k = 2 scale / (3B)
    }
    loss_term = 0.0f;
    return k * dr * dydz;            // k = scale
}

}  // namespace

// One workgroup of 4 waves processes rounds of 64 samples.  Phase 1: each wave runs one
// 16-sample tile forward (the first layer reads all 160 features) and backward with the
// transposed packed weights, keeping activations and deltas in registers, and stages them in
// LDS as [neuron][sample].  Phase 2: each wave owns a fixed set of 16x16 weight-gradient tiles
// (a quarter of every layer's column tiles) held in registers across rounds, and adds the
// round's 64 samples with MFMAs whose K dimension is the sample index.  At the end every tile is
// written once into this workgroup's partial gradient (canonical layout).
// PLAIN: targets given, relative L2 of eq. 12, no residual-variance mean, exp outputs (the general
// loss arithmetic compiled out).
template <int W, bool PLAIN = false>
__global__ __launch_bounds__(kTrainWaves * 64) void k_grad_f32(Points pts, Queries q,
                                                               const float *__restrict__ packed,
                                                               TrainArgs args, float *__restrict__ partials,
                                                               float *__restrict__ loss_partials) {
    static_assert(W == 64, "gradient kernel is laid out for width 64");
    constexpr F32Layout L{W};
    constexpr int MT = W / 16, KQ = W / 16;
    using S = GradLds<W>;
    __shared__ f32x4 smem4[(S::kTotal + 3) / 4];
    float *smem = (float *)smem4;
    float *sH = smem;
    float *sD = sH + S::kH;
    float *sD5 = sD + S::kD;
    float *sX = sD5 + S::kD5;
    float *sLoss = sX + S::kX;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t B = q.count;
    const bool use_loss = PLAIN || args.target != nullptr;
    const float kscale = use_loss ? 2.0f * args.loss_scale / (3.0f * (float)B) : args.loss_scale;

    // owned gradient tiles: first layer input columns {wave, wave+4, wave+8} (< 10), column tile
    // `wave` of W2..W4 and of W5
    f32x4 g1[3][MT], gh[3][MT], g5;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            g1[a][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
            gh[a][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
    g5 = f32x4{0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.0f;

    const int64_t n_chunks = (B + kChunk - 1) / kChunk;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        // ---------------- phase 1: forward + backward of this wave's 16 samples
        {
            const float *pk = opaque(packed);
            const int s = 16 * wave + col;   // sample slot in the chunk
            const int64_t b = chunk * kChunk + s;
            const bool valid = b < B;
            const int64_t bi = valid ? b : B - 1;
            const int64_t p = query_point(q, pts, bi);
            const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
            const float ws[3] = {q.wx[bi], q.wy[bi], q.wz[bi]};
            if (g == 0) {
                float *x = sX + s * kInputs;
                x[0] = xs[0]; x[1] = xs[1]; x[2] = xs[2];
                x[3] = ws[0]; x[4] = ws[1]; x[5] = ws[2];
                x[6] = xs[3]; x[7] = xs[4]; x[8] = xs[5]; x[9] = xs[6];
            }
            f32x4 h[4][MT];   // h1..h4
            {
                f32x4 a1[1][MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a1[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                layer1_surface<W>(a1[0], pk + L.offset(SEC_S), xs, lane, g);
                float dx[1] = {ws[0]}, dy[1] = {ws[1]}, dz[1] = {ws[2]};
                layer1_direction<W, 1>(a1, pk + L.offset(SEC_D), dx, dy, dz, lane, g);
                relu_all<W, 1>(a1);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[0][mt] = a1[0][mt];
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const float *sec = pk + L.offset(SEC_H0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], h[l - 1][kq][kk], o[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[l][mt][i] = relu_f32(o[mt][i]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const float *sec = pk + L.offset(SEC_O);
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    const f32x4 a = *(const f32x4 *)(sec + (kq * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) z5 = mfma4(a[kk], h[3][kq][kk], z5);
                }
            }
            // output delta: rows 0..2 live in lanes 0..15; everything else is zero
            f32x4 d5 = f32x4{0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float t = use_loss ? args.target[3 * b + c] : 0.0f;
                    const float dr = use_loss ? 0.0f : args.d_rgb[3 * b + c];
                    float lt;
                    d5[c] = PLAIN ? out_grad(z5[c], t, 0.0f, true, args.loss_eps, kscale, true, 0.0f, false, lt)
                                  : out_grad(z5[c], t, dr, use_loss, args.loss_eps, kscale,
                                             args.loss_kind == NIRC_LOSS_REL_L2, args.fr ? args.fr[c] : 0.0f,
                                             args.sig != 0, lt);
                    loss_acc += lt;
                }
            }
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sD5[c * kStride + s] = d5[c];
            }
            // stage activations
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        sH[(l * W + 16 * mt + 4 * g + i) * kStride + s] = h[l][mt][i];
            // backward: delta4 = (W5^T d5) .* [h4 > 0], then through W4^T, W3^T, W2^T
            f32x4 d[MT];
            {
                const float *sec = pk + L.offset(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 a = *(const f32x4 *)(sec + (mt * 64 + lane) * 4);
                    f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) o = mfma4(a[kk], d5[kk], o);
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[mt][i] = h[3][mt][i] > 0.0f ? o[i] : 0.0f;
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) sD[(3 * W + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
#pragma unroll
            for (int l = 3; l >= 1; --l) {   // delta_l = (W_{l+1}^T delta_{l+1}) .* [h_l > 0]
                const float *sec = pk + L.offset(SEC_T0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], d[kq][kk], o[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d[mt][i] = h[l - 1][mt][i] > 0.0f ? o[mt][i] : 0.0f;
                        sD[((l - 1) * W + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
                    }
            }
        }
        __syncthreads();
        // ---------------- phase 2: owned gradient tiles += staged deltas x activations
        // K position (step kk, lane group g) of sample group sq <-> sample 16 sq + 4 g + kk
#pragma unroll 1
        for (int sq = 0; sq < kChunk / 16; ++sq) {
            const int s0 = 16 * sq + 4 * g;
            // hidden layers W2..W4 (a = 0..2) and the output layer: column tile `wave`
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const f32x4 bv = *(const f32x4 *)(sH + (a * W + 16 * wave + col) * kStride + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 av = *(const f32x4 *)(sD + ((a + 1) * W + 16 * mt + col) * kStride + s0);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) gh[a][mt] = mfma4(av[kk], bv[kk], gh[a][mt]);
                }
            }
            {
                const f32x4 bv = *(const f32x4 *)(sH + (3 * W + 16 * wave + col) * kStride + s0);
                f32x4 av = f32x4{0.f, 0.f, 0.f, 0.f};
                if (col < 3) av = *(const f32x4 *)(sD5 + col * kStride + s0);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) g5 = mfma4(av[kk], bv[kk], g5);
            }
            // first layer: column tile = input index; features recomputed from staged inputs
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int input = wave + 4 * a;
                if (input >= kInputs) break;
                const int k = col >> 1, sc = col & 1;
                float bv[4];
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) {
                    float sn, cs;
                    enc_pair(sX[(s0 + kk) * kInputs + input], k, sn, cs);
                    bv[kk] = sc ? cs : sn;
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 av = *(const f32x4 *)(sD + (16 * mt + col) * kStride + s0);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) g1[a][mt] = mfma4(av[kk], bv[kk], g1[a][mt]);
                }
            }
        }
        __syncthreads();
    }

    // ---------------- write this workgroup's partial gradient (every entry exactly once)
    float *out = partials + (int64_t)blockIdx.x * n_params(W);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const int input = wave + 4 * a;
        if (input >= kInputs) break;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[w_offset(W, 0) + (int64_t)(16 * mt + 4 * g + i) * kFeat + 16 * input + col] = g1[a][mt][i];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[w_offset(W, 1 + a) + (int64_t)(16 * mt + 4 * g + i) * W + 16 * wave + col] = gh[a][mt][i];
    if (g == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) out[w_offset(W, 4) + (int64_t)i * W + 16 * wave + col] = g5[i];
    }
    // loss partial: fixed-order wave sum, then waves in order
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) loss_acc += __shfl_xor(loss_acc, d, 64);
    if (lane == 0) sLoss[wave] = loss_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kTrainWaves; ++w) t += sLoss[w];
        loss_partials[blockIdx.x] = t;
    }
}

// ------------------------------------------------------------------------------------------
// Width 128 (FP32).  Neither the weight-gradient tiles (280 of 16 x 16) nor the staged rows of
// all layers (278 KB) fit one pass, so the batch is swept three times; each sweep recomputes the
// forward and backward of every sample, stages only the rows its tiles need and owns a disjoint
// set of tiles (wave w: column tiles 2w, 2w + 1, or inputs w, w + 4, w + 8):
//   sweep 0: W2, W3    (rows h1, h2, delta2, delta3)
//   sweep 1: W4, W5    (rows h3, h4, delta4, output delta)
//   sweep 2: W1 + loss (rows delta1; features recomputed from the staged raw inputs)
template <int W>
struct GradWideLds {
    static constexpr int kRows = 4 * W + 4;                       // largest sweep
    static constexpr int kTotal = kRows * kStride + kChunk * kInputs;
};

template <int W, int SWEEP>
__global__ __launch_bounds__(kTrainWaves * 64) void k_grad_f32_wide(Points pts, Queries q,
                                                                    const float *__restrict__ packed, TrainArgs args,
                                                                    float *__restrict__ partials,
                                                                    float *__restrict__ loss_partials) {
    static_assert(W == 128, "wide gradient kernel");
    constexpr F32Layout L{W};
    constexpr int MT = W / 16, KQ = W / 16;
    using S = GradWideLds<W>;
    __shared__ f32x4 smem4[(S::kTotal + 3) / 4];
    __shared__ float sLoss[kTrainWaves];
    float *smem = (float *)smem4;
    float *rows = smem;                          // staged rows [row][sample]
    float *sX = smem + S::kRows * kStride;       // raw inputs [sample][10] (sweep 2)
    // row bases: sweep 0: h1 0, h2 W, delta2 2W, delta3 3W; sweep 1: h3 0, h4 W, delta4 2W,
    // d5 3W (4 rows); sweep 2: delta1 0
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t B = q.count;
    const bool use_loss = args.target != nullptr;
    const float kscale = use_loss ? 2.0f * args.loss_scale / (3.0f * (float)B) : args.loss_scale;

    constexpr int NACC = SWEEP == 0 ? 2 * 2 * MT : SWEEP == 1 ? 2 * MT + 2 : 3 * MT;
    f32x4 acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.0f;

    const int64_t n_chunks = (B + kChunk - 1) / kChunk;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        {
            const float *pk = opaque(packed);
            const int s = 16 * wave + col;
            const int64_t b = chunk * kChunk + s;
            const bool valid = b < B;
            const int64_t bi = valid ? b : B - 1;
            const int64_t p = query_point(q, pts, bi);
            const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
            const float ws[3] = {q.wx[bi], q.wy[bi], q.wz[bi]};
            if (SWEEP == 2 && g == 0) {
                float *x = sX + s * kInputs;
                x[0] = xs[0]; x[1] = xs[1]; x[2] = xs[2];
                x[3] = ws[0]; x[4] = ws[1]; x[5] = ws[2];
                x[6] = xs[3]; x[7] = xs[4]; x[8] = xs[5]; x[9] = xs[6];
            }
            f32x4 h[4][MT];
            {
                f32x4 a1[1][MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) a1[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                layer1_surface<W>(a1[0], pk + L.offset(SEC_S), xs, lane, g);
                float dx[1] = {ws[0]}, dy[1] = {ws[1]}, dz[1] = {ws[2]};
                layer1_direction<W, 1>(a1, pk + L.offset(SEC_D), dx, dy, dz, lane, g);
                relu_all<W, 1>(a1);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[0][mt] = a1[0][mt];
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const float *sec = pk + L.offset(SEC_H0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], h[l - 1][kq][kk], o[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[l][mt][i] = relu_f32(o[mt][i]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const float *sec = pk + L.offset(SEC_O);
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    const f32x4 a = *(const f32x4 *)(sec + (kq * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) z5 = mfma4(a[kk], h[3][kq][kk], z5);
                }
            }
            f32x4 d5 = f32x4{0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float t = use_loss ? args.target[3 * b + c] : 0.0f;
                    const float dr = use_loss ? 0.0f : args.d_rgb[3 * b + c];
                    float lt;
                    d5[c] = out_grad(z5[c], t, dr, use_loss, args.loss_eps, kscale, args.loss_kind == NIRC_LOSS_REL_L2,
                                     args.fr ? args.fr[c] : 0.0f, args.sig != 0, lt);
                    loss_acc += lt;
                }
            }
            // stage the activations this sweep needs
#pragma unroll
            for (int l = 0; l < 4; ++l) {
                const int base = SWEEP == 0 ? (l < 2 ? l * W : -1) : SWEEP == 1 ? (l >= 2 ? (l - 2) * W : -1) : -1;
                if (base < 0) continue;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) rows[(base + 16 * mt + 4 * g + i) * kStride + s] = h[l][mt][i];
            }
            if (SWEEP == 1 && g == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) rows[(3 * W + c) * kStride + s] = d5[c];
            }
            // backward: delta4 = (W5^T d5) .* [h4 > 0], then through W4^T, W3^T, W2^T
            f32x4 d[MT];
            {
                const float *sec = pk + L.offset(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 a = *(const f32x4 *)(sec + (mt * 64 + lane) * 4);
                    f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) o = mfma4(a[kk], d5[kk], o);
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[mt][i] = h[3][mt][i] > 0.0f ? o[i] : 0.0f;
                }
            }
            if (SWEEP == 1) {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) rows[(2 * W + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
            }
#pragma unroll
            for (int l = 3; l >= 1; --l) {   // delta_l = (W_{l+1}^T delta_{l+1}) .* [h_l > 0]
                const float *sec = pk + L.offset(SEC_T0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], d[kq][kk], o[mt]);
                }
                // delta_l rows: sweep 0 keeps delta2 (l = 2) at 2W and delta3 (l = 3) at 3W; sweep 2
                // keeps delta1 (l = 1) at 0
                const int base = SWEEP == 0 ? (l >= 2 ? l * W : -1) : SWEEP == 2 ? (l == 1 ? 0 : -1) : -1;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d[mt][i] = h[l - 1][mt][i] > 0.0f ? o[mt][i] : 0.0f;
                        if (base >= 0) rows[(base + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
                    }
            }
        }
        __syncthreads();
        // phase 2: K position (step kk, lane group g) of sample group sq <-> sample 16 sq + 4 g + kk
#pragma unroll 1
        for (int sq = 0; sq < kChunk / 16; ++sq) {
            const int s0 = 16 * sq + 4 * g;
            if constexpr (SWEEP == 0) {
                // W2 = delta2 h1^T (rows 2W, 0), W3 = delta3 h2^T (rows 3W, W)
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        const int ct = 2 * wave + cc;
                        const f32x4 bv = *(const f32x4 *)(rows + (a * W + 16 * ct + col) * kStride + s0);
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const f32x4 av = *(const f32x4 *)(rows + ((2 + a) * W + 16 * mt + col) * kStride + s0);
                            f32x4 &c = acc[(a * 2 + cc) * MT + mt];
#pragma unroll
                            for (int kk = 0; kk < 4; ++kk) c = mfma4(av[kk], bv[kk], c);
                        }
                    }
            } else if constexpr (SWEEP == 1) {
                // W4 = delta4 h3^T (rows 2W, 0), W5 = d5 h4^T (rows 3W, W)
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const int ct = 2 * wave + cc;
                    const f32x4 bv = *(const f32x4 *)(rows + (16 * ct + col) * kStride + s0);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const f32x4 av = *(const f32x4 *)(rows + (2 * W + 16 * mt + col) * kStride + s0);
                        f32x4 &c = acc[cc * MT + mt];
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) c = mfma4(av[kk], bv[kk], c);
                    }
                    const f32x4 b4 = *(const f32x4 *)(rows + (W + 16 * ct + col) * kStride + s0);
                    f32x4 a5 = f32x4{0.f, 0.f, 0.f, 0.f};
                    if (col < 3) a5 = *(const f32x4 *)(rows + (3 * W + col) * kStride + s0);
                    f32x4 &c5 = acc[2 * MT + cc];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) c5 = mfma4(a5[kk], b4[kk], c5);
                }
            } else {
                // W1 = delta1 e^T: column tile = input index, features recomputed from raw inputs
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int input = wave + 4 * a;
                    if (input >= kInputs) break;
                    const int k = col >> 1, sc = col & 1;
                    float bv[4];
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) {
                        float sn, cs;
                        enc_pair(sX[(s0 + kk) * kInputs + input], k, sn, cs);
                        bv[kk] = sc ? cs : sn;
                    }
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const f32x4 av = *(const f32x4 *)(rows + (16 * mt + col) * kStride + s0);
                        f32x4 &c = acc[a * MT + mt];
#pragma unroll
                        for (int kk = 0; kk < 4; ++kk) c = mfma4(av[kk], bv[kk], c);
                    }
                }
            }
        }
        __syncthreads();
    }

    float *out = partials + (int64_t)blockIdx.x * n_params(W);
    if constexpr (SWEEP == 0) {
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        out[w_offset(W, 1 + a) + (int64_t)(16 * mt + 4 * g + i) * W + 16 * (2 * wave + cc) + col] =
                            acc[(a * 2 + cc) * MT + mt][i];
    } else if constexpr (SWEEP == 1) {
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) {
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    out[w_offset(W, 3) + (int64_t)(16 * mt + 4 * g + i) * W + 16 * (2 * wave + cc) + col] =
                        acc[cc * MT + mt][i];
            if (g == 0) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    out[w_offset(W, 4) + (int64_t)i * W + 16 * (2 * wave + cc) + col] = acc[2 * MT + cc][i];
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int input = wave + 4 * a;
            if (input >= kInputs) break;
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    out[w_offset(W, 0) + (int64_t)(16 * mt + 4 * g + i) * kFeat + 16 * input + col] = acc[a * MT + mt][i];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) loss_acc += __shfl_xor(loss_acc, d, 64);
        if (lane == 0) sLoss[wave] = loss_acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int w = 0; w < kTrainWaves; ++w) t += sLoss[w];
            loss_partials[blockIdx.x] = t;
        }
    }
}

// grad[i] = inv_scale * sum_blk partials[blk][i] in a fixed order: a block handles 64 parameters
// (one per lane) with 16 waves; wave w sums the w-th sixteenth of the partials with eight running
// sums, then the sixteen wave sums are added in a fixed tree.  Raises `bad` on a non-finite
// entry.  Block 0 also reduces the loss.
constexpr int kReduceWaves = 16;

__device__ __forceinline__ void reduce_grad_block(const float *__restrict__ partials,
                                                  const float *__restrict__ loss_partials, int nblocks, int64_t np,
                                                  float inv_scale, float loss_norm, float *__restrict__ grad,
                                                  float *__restrict__ loss, uint32_t *bad, int blk,
                                                  float (*q)[64], const float *dyn_scale, float dyn_batch) {
    if (dyn_scale) inv_scale = 1.0f / (*dyn_scale * dyn_batch);
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blk * 64 + lane;
    const int per = (nblocks + kReduceWaves - 1) / kReduceWaves;
    const int b0 = min(nblocks, wave * per), b1 = min(nblocks, b0 + per);
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (i < np) {
        int b = b0;
        for (; b + 8 <= b1; b += 8)
#pragma unroll
            for (int u = 0; u < 8; ++u) acc[u] += partials[(int64_t)(b + u) * np + i];
        for (int u = 0; b < b1; ++b, ++u) acc[u] += partials[(int64_t)b * np + i];
    }
    q[wave][lane] = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    __syncthreads();
    if (wave == 0 && i < np) {
        float t[kReduceWaves / 2];
#pragma unroll
        for (int k = 0; k < kReduceWaves / 2; ++k) t[k] = q[2 * k][lane] + q[2 * k + 1][lane];
        const float sum = ((t[0] + t[1]) + (t[2] + t[3])) + ((t[4] + t[5]) + (t[6] + t[7]));
        const float gi = sum * inv_scale;
        grad[i] = gi;
        if (bad && !isfinite(gi)) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
    }
    // the loss: lane-strided sums of the partials, then a fixed shuffle tree (one wave, so the
    // loads are in flight together rather than one dependent load per partial)
    if (blk == 0 && wave == 0) {
        float t = 0.0f;
        for (int b = lane; b < nblocks; b += 64) t += loss_partials[b];
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) t += __shfl_xor(t, d, 64);
        if (lane == 0) {
            t *= loss_norm;
            if (loss) loss[0] = t;
            if (bad && !isfinite(t)) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
        }
    }
}

__global__ __launch_bounds__(kReduceWaves * 64) void k_reduce_grad(const float *__restrict__ partials,
                                                                   const float *__restrict__ loss_partials,
                                                                   int nblocks, int64_t np, float inv_scale,
                                                                   float loss_norm, float *__restrict__ grad,
                                                                   float *__restrict__ loss, uint32_t *bad,
                                                                   const float *dyn_scale, float dyn_batch) {
    __shared__ float q[kReduceWaves][64];
    reduce_grad_block(partials, loss_partials, nblocks, np, inv_scale, loss_norm, grad, loss, bad, blockIdx.x, q,
                      dyn_scale, dyn_batch);
}

// The reduction of every request of a training work list (request blockIdx.y), with the scale
// factors each request's own step uses (16-bit models: loss_scale * B).
__global__ __launch_bounds__(kReduceWaves * 64) void k_reduce_grad_multi(const TrainDesc *__restrict__ desc) {
    __shared__ float q[kReduceWaves][64];
    if ((int)blockIdx.y >= desc->n) return;
    const TrainReq &t = desc->req[blockIdx.y];
    const int64_t np = n_params(desc->width);
    if ((int64_t)blockIdx.x * 64 >= np) return;
    const float scale = t.loss_scale * (float)t.batch;
    reduce_grad_block(t.partials, t.lpart, t.nb, np, 1.0f / scale, 1.0f / (3.0f * (float)t.batch), t.grad, t.loss,
                      t.bad, blockIdx.x, q, t.dyn_scale, (float)t.batch);
}

__global__ void k_check_finite(const float *__restrict__ grad, int64_t np, uint32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np && !isfinite(grad[i])) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
}

// Adam (Kingma & Ba) with bias correction, t = step + 1; skipped entirely when `bad` is set.
__device__ __forceinline__ void adam_elem(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                                          const float *__restrict__ grad, const int64_t *step, const uint32_t *bad,
                                          int64_t np, float lr, float b1, float b2, float eps, int64_t i) {
    if (i >= np || *bad) return;
    const float t = (float)(*step + 1);
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    float mi = m[i], vi = v[i];
    w[i] = adam_update(w[i], mi, vi, grad[i], c1, c2, lr, b1, b2, eps);
    m[i] = mi;
    v[i] = vi;
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, const int64_t *step, const uint32_t *bad,
                       int64_t np, float lr, float b1, float b2, float eps) {
    adam_elem(w, m, v, grad, step, bad, np, lr, b1, b2, eps, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// Adam on the master weights with the FP32 packed copy refreshed in the same pass: thread i
// updates parameter i (the arithmetic of adam_elem) and stores it into the packed elements that
// hold it (f32_packed_targets; the zero padding is written once, when the weights are set).  A
// skipped step (`bad` set) changes nothing.  The last workgroup to finish (counted in `done`, zero
// between steps) commits the step or records its skip: every other workgroup has read `step` and
// `bad` before it counted itself.
template <int W>
__global__ __launch_bounds__(kAdamThreads) void k_adam_pack32(float *__restrict__ w, float *__restrict__ m,
                                                     float *__restrict__ v, const float *__restrict__ grad,
                                                     int64_t *step, uint32_t *flags, uint32_t *bad, uint32_t *done,
                                                     float *__restrict__ packed, float lr, float b1, float b2,
                                                     float eps) {
    constexpr int64_t np = n_params(W);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < np && *bad == 0u) {
        const float t = (float)(*step + 1);
        const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
        float mi = m[i], vi = v[i];
        const float wi = adam_update(w[i], mi, vi, grad[i], c1, c2, lr, b1, b2, eps);
        m[i] = mi;
        v[i] = vi;
        w[i] = wi;
        int e[2];
        const int n = f32_packed_targets(W, i, e);
        for (int k = 0; k < n; ++k) packed[e[k]] = wi;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(done, 1u) == gridDim.x - 1u) {
            __threadfence();
            commit_step(step, flags, bad, nullptr, nullptr);
            *done = 0u;
        }
    }
}

// ------------------------------------------------------------------------------------------

// Batch estimate of the residual's expectation per channel for the residual-variance loss:
// block b sums t - y over its contiguous share of the batch (each lane a strided run, then a
// fixed tree over the 256 lanes), and one wave adds the kFrBlocks block sums in a fixed tree.
// FP32 throughout; the order never depends on timing, so the result is deterministic.
__global__ __launch_bounds__(256) void k_residual_partials(const float *__restrict__ y, const float *__restrict__ t,
                                                           int64_t B, float *__restrict__ part) {
    __shared__ float sh[3][256];
    const int64_t per = (B + gridDim.x - 1) / gridDim.x;
    const int64_t b0 = (int64_t)blockIdx.x * per, b1 = min(B, b0 + per);
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += 256) {
        a0 += t[3 * b] - y[3 * b];
        a1 += t[3 * b + 1] - y[3 * b + 1];
        a2 += t[3 * b + 2] - y[3 * b + 2];
    }
    sh[0][threadIdx.x] = a0;
    sh[1][threadIdx.x] = a1;
    sh[2][threadIdx.x] = a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; ++c) sh[c][threadIdx.x] += sh[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[3 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_residual_final(const float *__restrict__ part, int64_t B,
                                                        float *__restrict__ fr) {
    static_assert(kFrBlocks == 256, "one lane per block sum");
    __shared__ float sh[3][256];
    const int i = threadIdx.x;
    for (int c = 0; c < 3; ++c) sh[c][i] = part[3 * i + c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (i < w)
            for (int c = 0; c < 3; ++c) sh[c][i] += sh[c][i + w];
        __syncthreads();
    }
    if (i < 3) fr[i] = sh[i][0] / (float)B;
}

hipError_t launch_residual_mean(const float *y, const float *t, int64_t B, float *part, float *fr, hipStream_t s) {
    if (B < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_residual_partials, dim3(kFrBlocks), dim3(256), 0, s, y, t, B, part);
    hipLaunchKernelGGL(k_residual_final, dim3(1), dim3(256), 0, s, part, B, fr);
    return hipGetLastError();
}

int train_blocks(int64_t batch) {
    int64_t chunks = (batch + kChunk - 1) / kChunk;
    if (chunks > kMaxResidentBlocks) chunks = kMaxResidentBlocks;
    return (int)(chunks < 1 ? 1 : chunks);
}

hipError_t launch_grad_partials(int W, const Points &pts, const Queries &q, const float *packed,
                                TrainArgs a, float *partials, float *loss_partials, int nblocks,
                                hipStream_t s) {
    if (W == 128) {
        const dim3 grid(nblocks), block(kTrainWaves * 64);
        hipLaunchKernelGGL((k_grad_f32_wide<128, 0>), grid, block, 0, s, pts, q, packed, a, partials, loss_partials);
        hipLaunchKernelGGL((k_grad_f32_wide<128, 1>), grid, block, 0, s, pts, q, packed, a, partials, loss_partials);
        hipLaunchKernelGGL((k_grad_f32_wide<128, 2>), grid, block, 0, s, pts, q, packed, a, partials, loss_partials);
        return hipGetLastError();
    }
    if (W != 64) return hipErrorInvalidValue;
    if (a.target && a.loss_kind == NIRC_LOSS_REL_L2 && !a.fr && !a.sig)
        hipLaunchKernelGGL((k_grad_f32<64, true>), dim3(nblocks), dim3(kTrainWaves * 64), 0, s, pts, q, packed, a,
                           partials, loss_partials);
    else
        hipLaunchKernelGGL((k_grad_f32<64>), dim3(nblocks), dim3(kTrainWaves * 64), 0, s, pts, q, packed, a,
                           partials, loss_partials);
    return hipGetLastError();
}

hipError_t launch_reduce_grad(int W, const float *partials, const float *loss_partials, int nblocks,
                              float inv_scale, float loss_norm, float *grad, float *loss,
                              uint32_t *bad, hipStream_t s, const float *dyn_scale, float dyn_batch) {
    const int64_t np = n_params(W);
    hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((np + 63) / 64)), dim3(kReduceWaves * 64), 0, s, partials,
                       loss_partials, nblocks, np, inv_scale, loss_norm, grad, loss, bad, dyn_scale, dyn_batch);
    return hipGetLastError();
}

hipError_t launch_check_finite(int W, const float *grad, uint32_t *bad, hipStream_t s) {
    const int64_t np = n_params(W);
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, grad, np, bad);
    return hipGetLastError();
}

hipError_t launch_adam(int W, float *master, float *m, float *v, const float *grad, int64_t *step,
                       uint32_t *flags, uint32_t *bad, float lr, float b1, float b2, float eps,
                       float *packed, uint16_t *packed16, int prec, hipStream_t s, uint32_t *done,
                       float *dyn_scale, uint32_t *good_steps) {
    const int64_t np = n_params(W);
    if (packed16)
        return launch_adam_pack16(W, prec, master, m, v, grad, step, flags, bad, dyn_scale, good_steps, done,
                                  packed16, lr, b1, b2, eps, s);
    const dim3 grid((unsigned)((np + kAdamThreads - 1) / kAdamThreads)), block(kAdamThreads);
    if (W == 64)
        hipLaunchKernelGGL(k_adam_pack32<64>, grid, block, 0, s, master, m, v, grad, step, flags, bad, done, packed,
                           lr, b1, b2, eps);
    else if (W == 128)
        hipLaunchKernelGGL(k_adam_pack32<128>, grid, block, 0, s, master, m, v, grad, step, flags, bad, done,
                           packed, lr, b1, b2, eps);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_reduce_grad_multi(const TrainDesc *desc, int W, hipStream_t s) {
    const int64_t np = n_params(W);
    hipLaunchKernelGGL(k_reduce_grad_multi, dim3((unsigned)((np + 63) / 64), kBatchMaxRequests),
                       dim3(kReduceWaves * 64), 0, s, desc);
    return hipGetLastError();
}

// Explicit-length variants (the hash-grid model's parameter vector).
hipError_t launch_reduce_grad_n(int64_t np, const float *partials, const float *loss_partials, int nblocks,
                                float inv_scale, float loss_norm, float *grad, float *loss, uint32_t *bad,
                                hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_grad, dim3((unsigned)((np + 63) / 64)), dim3(kReduceWaves * 64), 0, s, partials,
                       loss_partials, nblocks, np, inv_scale, loss_norm, grad, loss, bad, (const float *)nullptr, 1.0f);
    return hipGetLastError();
}

hipError_t launch_check_finite_n(int64_t np, const float *grad, uint32_t *bad, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, grad, np, bad);
    return hipGetLastError();
}

// k_adam over four consecutive elements per thread with 16-byte loads and stores (the long
// parameter vectors of the hash-grid model: one streaming pass over w, m, v and the gradient);
// the same arithmetic per element, and element by element in a ragged last group.
__global__ void k_adam4(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                        const float *__restrict__ grad, const int64_t *step, const uint32_t *bad, int64_t np,
                        float lr, float b1, float b2, float eps) {
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= np || *bad) return;
    const float t = (float)(*step + 1);
    const float c1 = 1.0f - powf(b1, t), c2 = 1.0f - powf(b2, t);
    if (i0 + 4 <= np) {
        const f32x4 g4 = *(const f32x4 *)(grad + i0);
        f32x4 m4 = *(const f32x4 *)(m + i0), v4 = *(const f32x4 *)(v + i0), w4 = *(const f32x4 *)(w + i0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float mk = m4[k], vk = v4[k];
            w4[k] = adam_update(w4[k], mk, vk, g4[k], c1, c2, lr, b1, b2, eps);
            m4[k] = mk;
            v4[k] = vk;
        }
        *(f32x4 *)(m + i0) = m4;
        *(f32x4 *)(v + i0) = v4;
        *(f32x4 *)(w + i0) = w4;
        return;
    }
    for (int64_t i = i0; i < np; ++i) {
        float mi = m[i], vi = v[i];
        w[i] = adam_update(w[i], mi, vi, grad[i], c1, c2, lr, b1, b2, eps);
        m[i] = mi;
        v[i] = vi;
    }
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

hipError_t launch_adam_n(int64_t np, float *master, float *m, float *v, const float *grad, const int64_t *step,
                         const uint32_t *bad, float lr, float b1, float b2, float eps, hipStream_t s) {
    if (aligned16(master) && aligned16(m) && aligned16(v) && aligned16(grad)) {
        const int64_t groups = (np + 3) / 4;
        hipLaunchKernelGGL(k_adam4, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, master, m, v, grad, step,
                           bad, np, lr, b1, b2, eps);
    } else {
        hipLaunchKernelGGL(k_adam, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, master, m, v, grad, step, bad,
                           np, lr, b1, b2, eps);
    }
    return hipGetLastError();
}

// g[i] *= scale, raising `bad` on a non-finite result.
__global__ void k_scale_check(float *__restrict__ g, int64_t n, float scale, uint32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float v = g[i] * scale;
        g[i] = v;
        if (bad && !isfinite(v)) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
    }
}

// Four elements per thread with 16-byte accesses where the buffer allows it.
__global__ void k_scale_check4(float *__restrict__ g, int64_t n, float scale, uint32_t *bad) {
    const int64_t i0 = 4 * ((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
    if (i0 >= n) return;
    bool fin = true;
    if (i0 + 4 <= n) {
        f32x4 x = *(const f32x4 *)(g + i0);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            x[k] *= scale;
            fin = fin && isfinite(x[k]);
        }
        *(f32x4 *)(g + i0) = x;
    } else {
        for (int64_t i = i0; i < n; ++i) {
            const float x = g[i] * scale;
            g[i] = x;
            fin = fin && isfinite(x);
        }
    }
    if (bad && !fin) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
}

__global__ void k_grid_acc_finish(const unsigned long long *__restrict__ acc, const uint32_t *__restrict__ nonfinite,
                                  float *__restrict__ g, int64_t n, float scale, uint32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float v = *nonfinite ? __builtin_nanf("") : __ll2float_rn((long long)acc[i]) * 0x1p-36f * scale;
    g[i] = v;
    if (bad && !isfinite(v)) atomicOr(bad, NIRC_FLAG_NONFINITE_GRAD);
}

hipError_t launch_grid_acc_finish(const GridAcc &ga, float *grad, int64_t n, float scale, uint32_t *bad,
                                  hipStream_t s) {
    static_assert(kGridFix == 36, "the finish kernel scales by 2^-36");
    hipLaunchKernelGGL(k_grid_acc_finish, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ga.acc, ga.nonfinite,
                       grad, n, scale, bad);
    return hipGetLastError();
}

hipError_t launch_scale_check(float *g, int64_t n, float scale, uint32_t *bad, hipStream_t s) {
    if (aligned16(g)) {
        const int64_t groups = (n + 3) / 4;
        hipLaunchKernelGGL(k_scale_check4, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, s, g, n, scale, bad);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(k_scale_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, n, scale, bad);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// The hash-grid model in FP32 (width 64): k_grad_f32's two phases with the 64 grid / SH / phi
// inputs staged as rows [canonical input][sample] for the first layer's weight gradient.  Each
// sample's gradient with respect to its 24 grid values (W1_grid^T delta1, from the transposed
// TS32 section) is kept in registers through phase 2 and then scattered into the grid-entry
// gradient by 64-bit fixed-point integer atomic adds (grid_acc_add; the 16 values of one
// (sample, level) in 16 consecutive lanes, x neighbours in adjacent lane pairs, zero values
// skipped), staged through LDS that phase 2 has released.
namespace {
constexpr int kScatRow32 = 28;   // per sample: 24 grid-value gradients, position, pad
struct HashGrad32Lds {
    static constexpr int kH = 4 * 64 * kStride;
    static constexpr int kD = 4 * 64 * kStride;
    static constexpr int kD5 = 4 * kStride;
    static constexpr int kE = kHashIn * kStride;
    static constexpr int kTotal = kH + kD + kD5 + kE;
    static_assert(kTrainWaves * 16 * kScatRow32 <= kH, "scatter staging reuses the activation rows");
};
}  // namespace

__global__ __launch_bounds__(kTrainWaves * 64) void k_hash_grad_f32(Points pts, Queries q,
                                                                    const float *__restrict__ packed,
                                                                    const float2 *__restrict__ table,
                                                                    HashGridArgs grid, TrainArgs args,
                                                                    float *__restrict__ partials,
                                                                    float *__restrict__ loss_partials,
                                                                    GridAcc gacc) {
    constexpr int W = 64, MT = 4, KQ = 4;
    using S = HashGrad32Lds;
    __shared__ f32x4 smem4[(S::kTotal + 3) / 4];
    __shared__ float sLoss[kTrainWaves];
    __shared__ HashLevel s_lv[kHashLevels];
    float *smem = (float *)smem4;
    float *sH = smem;
    float *sD = sH + S::kH;
    float *sD5 = sD + S::kD;
    float *sE = sD5 + S::kD5;
    stage_levels(s_lv, grid);
    __syncthreads();

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t B = q.count;
    const bool rel = args.loss_kind == NIRC_LOSS_REL_L2;
    // the host passes loss_scale * B: k = 2 loss_scale / 3 per sample
    const float kscale = 2.0f * args.loss_scale / (3.0f * (float)B);

    f32x4 g1[MT], gh[3][MT], g5;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        g1[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int a = 0; a < 3; ++a) gh[a][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
    g5 = f32x4{0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.0f;

    const int64_t n_chunks = (B + kChunk - 1) / kChunk;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        // ---------------- phase 1: forward + backward of this wave's 16 samples
        f32x4 de[2];   // rows 16 m + 4 g + i of W1_grid^T delta1 (grid values 2 k + f of level k)
        float x0, x1, x2;
        bool valid;
        {
            const float *pk = opaque(packed);
            const int s = 16 * wave + col;
            const int64_t b = chunk * kChunk + s;
            valid = b < B;
            const int64_t bi = valid ? b : B - 1;
            const int64_t p = query_point(q, pts, bi);
            const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
            x0 = xs[0];
            x1 = xs[1];
            x2 = xs[2];
            float v[6], ph[4], sd[8];
            hash_values6(s_lv, grid.tmask, table, xs[0], xs[1], xs[2], g, v);
            hash_phi4(xs[3], xs[4], xs[5], xs[6], g, ph);
            hash_dir_values_f32(q.wx[bi], q.wy[bi], q.wz[bi], g, sd);
            // canonical input rows: grid 6 g + k, SH 24 + 4 k + g, phi 49 + 4 j + g
#pragma unroll
            for (int k = 0; k < 6; ++k) sE[(6 * g + k) * kStride + s] = v[k];
#pragma unroll
            for (int k = 0; k < 7; ++k)
                if (4 * k + g < 25) sE[(24 + 4 * k + g) * kStride + s] = sd[k];
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (4 * j + g < 15) sE[(49 + 4 * j + g) * kStride + s] = ph[j];

            f32x4 h[4][MT];
            {
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[0][mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                hash_layer1_surface_f32(h[0], pk, v, ph, lane);
                const float *gD = pk + kHash32S;
#pragma unroll
                for (int kq = 0; kq < 2; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(gD + ((mt * 2 + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) h[0][mt] = mfma4(a[mt][kk], sd[4 * kq + kk], h[0][mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[0][mt][i] = relu_f32(h[0][mt][i]);
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const float *sec = pk + hash_sec32(SEC_H0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], h[l - 1][kq][kk], o[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) h[l][mt][i] = relu_f32(o[mt][i]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const float *sec = pk + hash_sec32(SEC_O);
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    const f32x4 a = *(const f32x4 *)(sec + (kq * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) z5 = mfma4(a[kk], h[3][kq][kk], z5);
                }
            }
            f32x4 d5 = f32x4{0.f, 0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float lt;
                    d5[c] = out_grad(z5[c], args.target[3 * b + c], 0.0f, true, args.loss_eps, kscale, rel, 0.0f,
                                     false, lt);
                    loss_acc += lt;
                }
            }
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sD5[c * kStride + s] = d5[c];
            }
#pragma unroll
            for (int l = 0; l < 4; ++l)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        sH[(l * W + 16 * mt + 4 * g + i) * kStride + s] = h[l][mt][i];
            f32x4 d[MT];
            {
                const float *sec = pk + hash_sec32(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 a = *(const f32x4 *)(sec + (mt * 64 + lane) * 4);
                    f32x4 o = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) o = mfma4(a[kk], d5[kk], o);
#pragma unroll
                    for (int i = 0; i < 4; ++i) d[mt][i] = h[3][mt][i] > 0.0f ? o[i] : 0.0f;
                }
            }
#pragma unroll
            for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) sD[(3 * W + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
#pragma unroll
            for (int l = 3; l >= 1; --l) {
                const float *sec = pk + hash_sec32(SEC_T0 + (l - 1));
                f32x4 o[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) o[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    f32x4 a[MT];
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) a[mt] = *(const f32x4 *)(sec + ((mt * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk)
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) o[mt] = mfma4(a[mt][kk], d[kq][kk], o[mt]);
                }
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        d[mt][i] = h[l - 1][mt][i] > 0.0f ? o[mt][i] : 0.0f;
                        sD[((l - 1) * W + 16 * mt + 4 * g + i) * kStride + s] = d[mt][i];
                    }
            }
            // d = delta1; the grid-value gradient of this sample (column col)
            const float *sec = pk + kHash32TS;
#pragma unroll
            for (int m = 0; m < 2; ++m) {
                de[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kq = 0; kq < KQ; ++kq) {
                    const f32x4 a = *(const f32x4 *)(sec + ((m * KQ + kq) * 64 + lane) * 4);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) de[m] = mfma4(a[kk], d[kq][kk], de[m]);
                }
            }
        }
        __syncthreads();
        // ---------------- phase 2: owned weight-gradient tiles (W1: inputs 16 wave .. 16 wave + 15)
#pragma unroll 1
        for (int sq = 0; sq < kChunk / 16; ++sq) {
            const int s0 = 16 * sq + 4 * g;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const f32x4 bv = *(const f32x4 *)(sH + (a * W + 16 * wave + col) * kStride + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 av = *(const f32x4 *)(sD + ((a + 1) * W + 16 * mt + col) * kStride + s0);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) gh[a][mt] = mfma4(av[kk], bv[kk], gh[a][mt]);
                }
            }
            {
                const f32x4 bv = *(const f32x4 *)(sH + (3 * W + 16 * wave + col) * kStride + s0);
                f32x4 av = f32x4{0.f, 0.f, 0.f, 0.f};
                if (col < 3) av = *(const f32x4 *)(sD5 + col * kStride + s0);
#pragma unroll
                for (int kk = 0; kk < 4; ++kk) g5 = mfma4(av[kk], bv[kk], g5);
            }
            {
                const f32x4 bv = *(const f32x4 *)(sE + (16 * wave + col) * kStride + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const f32x4 av = *(const f32x4 *)(sD + (16 * mt + col) * kStride + s0);
#pragma unroll
                    for (int kk = 0; kk < 4; ++kk) g1[mt] = mfma4(av[kk], bv[kk], g1[mt]);
                }
            }
        }
        __syncthreads();
        // ---------------- scatter of the grid-value gradients (staging in the released rows)
        {
            float *sg = smem + wave * (16 * kScatRow32);
#pragma unroll
            for (int m = 0; m < 2; ++m)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * m + 4 * g + i;
                    if (k < 24) sg[col * kScatRow32 + k] = valid ? de[m][i] : 0.0f;
                }
            if (g == 0) {
                sg[col * kScatRow32 + 24] = x0;
                sg[col * kScatRow32 + 25] = x1;
                sg[col * kScatRow32 + 26] = x2;
            }
            wave_sync();
            const int qd = lane >> 4, corner = (lane & 15) >> 1, f = lane & 1;
#pragma unroll 4
            for (int it = 0; it < 16 * kHashLevels / 4; ++it) {
                const int pr = 4 * it + qd;
                const int smp = pr / kHashLevels, level = pr - kHashLevels * smp;
                const float *row = sg + smp * kScatRow32;
                const float dv = row[2 * level + f];
                const HashLevel lv = s_lv[level];
                const HashCell cell = hash_cell(row[24], row[25], row[26], lv.res);
                float w;
                const uint32_t e = hash_entry(lv, grid.tmask, cell, corner, w);
                grid_acc_add(gacc, 2 * (size_t)e + f, w * dv);
            }
        }
        __syncthreads();   // the next chunk's rows overwrite the staging
    }

    float *out = partials + (int64_t)blockIdx.x * kHashMlp;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int i = 0; i < 4; ++i) out[(int64_t)(16 * mt + 4 * g + i) * kHashIn + 16 * wave + col] = g1[mt][i];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int mt = 0; mt < MT; ++mt)
#pragma unroll
            for (int i = 0; i < 4; ++i)
                out[W * kHashIn + a * W * W + (int64_t)(16 * mt + 4 * g + i) * W + 16 * wave + col] = gh[a][mt][i];
    if (g == 0) {
#pragma unroll
        for (int i = 0; i < 3; ++i) out[W * kHashIn + 3 * W * W + (int64_t)i * W + 16 * wave + col] = g5[i];
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) loss_acc += __shfl_xor(loss_acc, d, 64);
    if (lane == 0) sLoss[wave] = loss_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kTrainWaves; ++w) t += sLoss[w];
        loss_partials[blockIdx.x] = t;
    }
}

hipError_t launch_hash_grad32(const Points &pts, const Queries &q, const float *packed, const float *table,
                              const HashGridArgs &grid, TrainArgs a, float *partials, float *loss_partials,
                              GridAcc gacc, int nblocks, hipStream_t s) {
    if (!a.target) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_hash_grad_f32, dim3(nblocks), dim3(kTrainWaves * 64), 0, s, pts, q, packed,
                       (const float2 *)table, grid, a, partials, loss_partials, gacc);
    return hipGetLastError();
}

}  // namespace nirc
