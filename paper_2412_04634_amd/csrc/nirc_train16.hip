// 16-bit training: fused forward + relative-L2 loss + backward to per-workgroup weight-gradient
// partials with BF16 / FP16 MFMA operands and FP32 accumulation.  Partials use the canonical
// layout of the FP32 kernel, so the fixed-order reduction and Adam (on the FP32 master weights)
// are shared.  The per-sample output gradient is not divided by the batch size inside the
// kernel (the host folds 1/B into the loss scale), which keeps every 16-bit delta near unit
// magnitude whatever the batch; the reduction divides the scale out again.
#include "nirc_hash.hpp"

namespace nirc {

namespace {

constexpr int kWaves16 = 4;
constexpr int kChunk16 = 16 * kWaves16;   // samples per round (two 32-sample K-blocks)
constexpr int kRow16 = kChunk16 + 8;      // LDS row stride in 16-bit elements (144 B)

template <int W>
struct Grad16Lds {
    static constexpr int kH = 4 * W * kRow16;    // h1..h4 (after ReLU)  [layer][neuron][sample]
    static constexpr int kD = 4 * W * kRow16;    // delta1..delta4       [layer][neuron][sample]
    static constexpr int kD5 = 4 * kRow16;       // output-layer delta, rows 0..3
    static constexpr int kE = kFeat * kRow16;    // input features      [canonical feature][sample]
    static constexpr int kTotal = kH + kD + kD5 + kE;   // 16-bit elements
};

template <int PREC>
__device__ __forceinline__ uint16_t to16(float x) {
    return (uint16_t)(pack2<PREC>(x, 0.0f) & 0xFFFFu);
}

// Packs two result tiles into a chained B operand without ReLU (backward deltas).
template <int PREC>
__device__ __forceinline__ u32x4 chain_plain(const f32x4 &lo, const f32x4 &hi) {
    return u32x4{pack2<PREC>(lo[0], lo[1]), pack2<PREC>(lo[2], lo[3]), pack2<PREC>(hi[0], hi[1]),
                 pack2<PREC>(hi[2], hi[3])};
}

// 16-bit element e of an operand (8 values in 4 dwords).
__device__ __forceinline__ uint16_t half_of(const u32x4 &v, int e) {
    return (uint16_t)((v[e >> 1] >> (16 * (e & 1))) & 0xFFFFu);
}

// Stores chained activations (B layout, lane (g, col): K position 8g + j of K-block kb is
// neuron 32 kb + 16 (j / 4) + 4 g + j % 4) as rows [neuron][sample].
template <int W>
__device__ __forceinline__ void stage_chain(uint16_t *rows, const u32x4 (&v)[W / 32], int g, int s) {
#pragma unroll
    for (int kb = 0; kb < W / 32; ++kb)
#pragma unroll
        for (int j = 0; j < 8; ++j) rows[chained_neuron16(kb, g, j) * kRow16 + s] = half_of(v[kb], j);
}

__device__ inline float out_grad16(float z, float t, float dr, bool use_loss, float eps, float k, bool rel, float fr,
                                   bool sig, float &loss_term) {
    const float y = sig ? logistic(z) : expf(z);
    const float dydz = sig ? y * (1.0f - y) : y;
    if (use_loss) {
        const float d = (y - t) + fr, den = rel ? y * y + eps : 1.0f;
        loss_term = d * d / den;
        return k * d / den * dydz;
    }
    loss_term = 0.0f;
    return k * dr * dydz;
}

// One sample's inputs to a training round: its point's attributes, its direction and its
// target (or output gradient).  Loaded ahead of use in two steps, so that neither the point
// index nor the attributes that depend on it are waited for: the query's own values one round
// ahead (load_query16), the point's attributes half a round ahead (load_point16).
struct Sample16 {
    float x[7], w[3], t[3];
    int64_t bi;   // the query (the batch's last one for the slots past its end)
    int64_t j;    // its point index as given (bi itself when the queries carry none)
    bool valid;
};

__device__ __forceinline__ void load_query16(const Queries &q, const TrainArgs &args, int64_t b, int64_t B,
                                             Sample16 &o) {
    o.valid = b < B;
    o.bi = o.valid ? b : B - 1;
    o.j = q.point ? (int64_t)q.point[o.bi] : o.bi;
    o.w[0] = q.wx[o.bi], o.w[1] = q.wy[o.bi], o.w[2] = q.wz[o.bi];
    const float *t = args.target ? args.target : args.d_rgb;
#pragma unroll
    for (int c = 0; c < 3; ++c) o.t[c] = t[3 * o.bi + c];
}

__device__ __forceinline__ void load_point16(const Points &pts, const Queries &q, Sample16 &o) {
    // the checks of query_point on the index loaded before
    int64_t p = o.j;
    if (p < 0 || p >= pts.count) {
        if (q.err) atomicOr(q.err, NIRC_FLAG_BAD_POINT_INDEX);
        p = p < 0 ? 0 : pts.count - 1;
    }
    o.x[0] = pts.px[p], o.x[1] = pts.py[p], o.x[2] = pts.pz[p];
    o.x[3] = pts.nx[p], o.x[4] = pts.ny[p], o.x[5] = pts.nz[p], o.x[6] = pts.rough[p];
}

}  // namespace

// One workgroup of 4 waves processes rounds of 64 samples.  Phase 1: each wave takes 16 samples
// through the 16-bit forward chain (packed weights read from global memory) and back through
// the transposed sections, and stages the ReLU outputs, the deltas and the input features as
// 16-bit rows [neuron][sample] in LDS (the ReLU masks come from the 16-bit activations).
// Phase 2: each wave owns the same weight-gradient tiles as in the FP32 kernel and adds the
// round with 16x16x32 MFMAs whose K dimension is the sample index.
// Block `blk` of `nblk` over the batch (chunks blk, blk + nblk, ...): its partial gradient goes to
// `out` [n_params], its loss partial to *loss_out.  smem: Grad16Lds<W>::kTotal 16-bit elements;
// sLoss: kWaves16 floats.  Ends after a workgroup barrier, so a caller may run the next block on
// the same LDS.  PLAIN: the caller guarantees the common case (targets given, relative L2 of
// eq. 12, no residual-variance mean, exp outputs), so the general loss arithmetic is compiled out.
template <int W, int PREC, bool PLAIN = false>
__device__ __forceinline__ void grad16_block(const Points &pts, const Queries &q, const uint16_t *packed,
                                             const TrainArgs &args, float *out, float *loss_out, int64_t blk,
                                             int64_t nblk, uint16_t *smem, float *sLoss) {
    static_assert(W == 64, "gradient kernel is laid out for width 64");
    constexpr H16Layout L{W};
    constexpr int MT = W / 16, KB = W / 32;
    using S = Grad16Lds<W>;
    uint16_t *sH = smem;
    uint16_t *sD = sH + S::kH;
    uint16_t *sD5 = sD + S::kD;
    uint16_t *sE = sD5 + S::kD5;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t B = q.count;
    const bool use_loss = PLAIN || args.target != nullptr;
    // the host passes loss_scale * B for 16-bit models (or the dynamic scale is taken times B):
    // k = 2 loss_scale / 3 per sample
    const float ls = args.dyn_scale ? *args.dyn_scale * (float)B : args.loss_scale;
    const float kscale = use_loss ? 2.0f * ls / (3.0f * (float)B) : ls;

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

    const int64_t n_chunks = (B + kChunk16 - 1) / kChunk16;
    const int s = 16 * wave + col;   // sample slot in the round
    Sample16 next;
    if (blk < n_chunks) {
        load_query16(q, args, blk * kChunk16 + s, B, next);
        load_point16(pts, q, next);
    }
    for (int64_t chunk = blk; chunk < n_chunks; chunk += nblk) {
        // ---------------- phase 1: forward + backward of this wave's 16 samples
        {
            const uint16_t *pk = opaque(packed);
            const Sample16 cur = next;
            const bool more = chunk + nblk < n_chunks;
            if (more) load_query16(q, args, (chunk + nblk) * kChunk16 + s, B, next);
            const bool valid = cur.valid;
            const float *xs = cur.x, *ws = cur.w;
            // scheduling fences between the steps of a round: left free, the compiler interleaves
            // the steps' loads and LDS stores in an order that measured a third slower
            __builtin_amdgcn_sched_barrier(0);

            // input features of frequencies 2g, 2g + 1: (sin, 2 cos) pairs for the MFMAs, and
            // (sin, cos) rows for the first layer's gradient
            float f[44];
#pragma unroll
            for (int i = 0; i < 7; ++i) enc_pair2_fast(xs[i], g, f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                enc_pair2_fast(ws[i], g, f[28 + 4 * i], f[29 + 4 * i], f[30 + 4 * i], f[31 + 4 * i]);
#pragma unroll
            for (int t = 0; t < 28; ++t)
                sE[feature_of(true, g, t) * kRow16 + s] = to16<PREC>((t & 1) ? 0.5f * f[t] : f[t]);
#pragma unroll
            for (int t = 0; t < 12; ++t)
                sE[feature_of(false, g, t) * kRow16 + s] = to16<PREC>((t & 1) ? 0.5f * f[28 + t] : f[28 + t]);
            __builtin_amdgcn_sched_barrier(0);

            // forward
            u32x4 hb[4][KB];   // h1..h4 after ReLU, as chained B operands
            {
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                const uint16_t *gS = pk + L.offset(SEC_S);
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const float *fk = f + 8 * kb;
                    const u32x4 bop = kb < 3 ? u32x4{pack2<PREC>(fk[0], fk[1]), pack2<PREC>(fk[2], fk[3]),
                                                     pack2<PREC>(fk[4], fk[5]), pack2<PREC>(fk[6], fk[7])}
                                             : u32x4{pack2<PREC>(fk[0], fk[1]), pack2<PREC>(fk[2], fk[3]), 0u, 0u};
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        h[mt] = mfma16<PREC>(*(const u32x4 *)(gS + ((mt * 4 + kb) * 64 + lane) * 8), bop, h[mt]);
                }
                const float *fd = f + 28;
                const u32x4 bd0 = {pack2<PREC>(fd[0], fd[1]), pack2<PREC>(fd[2], fd[3]), pack2<PREC>(fd[4], fd[5]),
                                   pack2<PREC>(fd[6], fd[7])};
                const u32x4 bd1 = {pack2<PREC>(fd[8], fd[9]), pack2<PREC>(fd[10], fd[11]), 0u, 0u};
                const uint16_t *gD = pk + L.offset(SEC_D);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    h[mt] = mfma16<PREC>(*(const u32x4 *)(gD + ((mt * 2 + 0) * 64 + lane) * 8), bd0, h[mt]);
                    h[mt] = mfma16<PREC>(*(const u32x4 *)(gD + ((mt * 2 + 1) * 64 + lane) * 8), bd1, h[mt]);
                }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[0][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const uint16_t *sec = pk + L.offset(SEC_H0 + (l - 1));
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        h[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), hb[l - 1][kb],
                                             h[mt]);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[l][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const uint16_t *sec = pk + L.offset(SEC_O);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    z5 = mfma16<PREC>(*(const u32x4 *)(sec + (kb * 64 + lane) * 8), hb[3][kb], z5);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (more) load_point16(pts, q, next);
#pragma unroll
            for (int l = 0; l < 4; ++l) stage_chain<W>(sH + l * W * kRow16, hb[l], g, s);

            // output delta (rows 0..2 in lanes 0..15)
            float d5[3] = {0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float t = use_loss ? cur.t[c] : 0.0f;
                    const float dr = use_loss ? 0.0f : cur.t[c];
                    float lt;
                    d5[c] = PLAIN ? out_grad16(z5[c], t, 0.0f, true, args.loss_eps, kscale, true, 0.0f, false, lt)
                                  : out_grad16(z5[c], t, dr, use_loss, args.loss_eps, kscale,
                                               args.loss_kind == NIRC_LOSS_REL_L2, args.fr ? args.fr[c] : 0.0f,
                                               args.sig != 0, lt);
                    loss_acc += lt;
                }
            }
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sD5[c * kRow16 + s] = to16<PREC>(c < 3 ? d5[c] : 0.0f);
            }

            // backward: delta4 = (W5^T d5) .* [h4 > 0]; OT holds output o at K position 8g + j
            // (j < 4, o = 4g + j), so only lane group 0 carries d5 in the B operand
            f32x4 dl[MT];
            {
                const u32x4 bop = g == 0 ? u32x4{pack2<PREC>(d5[0], d5[1]), pack2<PREC>(d5[2], 0.0f), 0u, 0u}
                                         : u32x4{0u, 0u, 0u, 0u};
                const uint16_t *sec = pk + L.offset(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + (mt * 64 + lane) * 8), bop, f32x4{0.f, 0.f, 0.f, 0.f});
            }
#pragma unroll
            for (int l = 3; l >= 0; --l) {
                // mask with [h_{l+1} > 0]: result row i of tile mt is chained position
                // (kb = mt / 2, j = 4 (mt % 2) + i) of hb[l]
                u32x4 db[KB];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint16_t hv = half_of(hb[l][mt >> 1], 4 * (mt & 1) + i);
                        if (hv == 0) dl[mt][i] = 0.0f;   // ReLU output is +0 exactly when inactive
                    }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) db[kb] = chain_plain<PREC>(dl[2 * kb], dl[2 * kb + 1]);
                stage_chain<W>(sD + l * W * kRow16, db, g, s);
                if (l == 0) break;
                // delta_l = (W_{l+1}^T delta_{l+1}) .* [h_l > 0]
                const uint16_t *sec = pk + L.offset(SEC_T0 + (l - 1));
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) dl[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), db[kb], dl[mt]);
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
        // ---------------- phase 2: owned gradient tiles += staged deltas x activations
        // K position 8g + j of K-block kb <-> sample 32 kb + 8 g + j
#pragma unroll
        for (int kb = 0; kb < kChunk16 / 32; ++kb) {
            const int s0 = 32 * kb + 8 * g;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const u32x4 bv = *(const u32x4 *)(sH + (a * W + 16 * wave + col) * kRow16 + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const u32x4 av = *(const u32x4 *)(sD + ((a + 1) * W + 16 * mt + col) * kRow16 + s0);
                    gh[a][mt] = mfma16<PREC>(av, bv, gh[a][mt]);
                }
            }
            {
                const u32x4 bv = *(const u32x4 *)(sH + (3 * W + 16 * wave + col) * kRow16 + s0);
                u32x4 av = u32x4{0u, 0u, 0u, 0u};
                if (col < 3) av = *(const u32x4 *)(sD5 + col * kRow16 + s0);
                g5 = mfma16<PREC>(av, bv, g5);
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int input = wave + 4 * a;
                if (input >= kInputs) break;
                const u32x4 bv = *(const u32x4 *)(sE + (16 * input + col) * kRow16 + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const u32x4 av = *(const u32x4 *)(sD + (16 * mt + col) * kRow16 + s0);
                    g1[a][mt] = mfma16<PREC>(av, bv, g1[a][mt]);
                }
            }
        }
        __builtin_amdgcn_sched_barrier(0);
        __syncthreads();
        __builtin_amdgcn_sched_barrier(0);
    }

    // ---------------- write this block's partial gradient (every entry exactly once)
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
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) loss_acc += __shfl_xor(loss_acc, d, 64);
    if (lane == 0) sLoss[wave] = loss_acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.0f;
        for (int w = 0; w < kWaves16; ++w) t += sLoss[w];
        *loss_out = t;
    }
    __syncthreads();
}

template <int W, int PREC, bool PLAIN = false>
__global__ __launch_bounds__(kWaves16 * 64) void k_grad_h16(Points pts, Queries q, const uint16_t *__restrict__ packed,
                                                            TrainArgs args, float *__restrict__ partials,
                                                            float *__restrict__ loss_partials) {
    __shared__ u32x4 smem4[(Grad16Lds<W>::kTotal + 7) / 8];
    __shared__ float sLoss[kWaves16];
    grad16_block<W, PREC, PLAIN>(pts, q, packed, args, partials + (int64_t)blockIdx.x * n_params(W),
                          loss_partials + blockIdx.x, blockIdx.x, gridDim.x, (uint16_t *)smem4, sLoss);
}

// The gradient step of several models at once (continuous batching of the streams' training
// passes): request r's workgroups are the virtual blocks vb0 .. vb0 + nb - 1 of the list, and a
// fixed grid walks the virtual blocks in order.  Virtual block b of a request computes exactly
// what block b of k_grad_h16 computes for that request alone (same chunks, same order), so the
// partials, and everything after them, are bit-identical.
template <int W, int PREC>
__global__ __launch_bounds__(kWaves16 * 64) void k_grad_h16_multi(const TrainDesc *__restrict__ desc) {
    __shared__ u32x4 smem4[(Grad16Lds<W>::kTotal + 7) / 8];
    __shared__ float sLoss[kWaves16];
    const int n = desc->n, total = desc->total_vb;
    for (int v = blockIdx.x; v < total; v += gridDim.x) {
        int r = 0;
        while (r + 1 < n && desc->req[r + 1].vb0 <= v) ++r;
        const TrainReq &t = desc->req[r];
        const int b = v - t.vb0;
        const Queries q{t.swx, t.swy, t.swz, t.sp, t.batch, t.bad};
        const TrainArgs a{t.stgt, nullptr, t.loss_eps, t.loss_scale * (float)t.batch, t.loss_kind, nullptr,
                          t.output == NIRC_OUTPUT_VISIBILITY, t.dyn_scale};
        grad16_block<W, PREC>(t.pts, q, t.packed16, a, t.partials + (int64_t)b * n_params(W), t.lpart + b, b, t.nb,
                              (uint16_t *)smem4, sLoss);
    }
}

// ------------------------------------------------------------------------------------------
// Width 128.  The weight gradient no longer fits in the registers of one workgroup pass (280
// tiles of 16 x 16), so the batch is swept twice, each sweep owning a disjoint set of tiles and
// recomputing the forward and backward of every sample:
//   sweep 0: W2, W3, W4 (wave w owns column tiles 2w, 2w + 1 of each, 48 tiles);
//   sweep 1: W1 (inputs w, w + 4, w + 8) and W5 (column tiles 2w, 2w + 1), and the loss.
// Each sweep stages in LDS only the rows its tiles need.  Weights are read from global memory.
template <int W>
struct Grad16WideLds {
    static constexpr int kRows0 = 6 * W;                  // sweep 0: h1..h3, delta2..delta4
    static constexpr int kRows1 = 2 * W + kFeat + 4;      // sweep 1: h4, delta1, features, d5
    static constexpr int kTotal = (kRows0 > kRows1 ? kRows0 : kRows1) * kRow16;   // 16-bit elements
};

template <int W, int PREC, int SWEEP>
__global__ __launch_bounds__(kWaves16 * 64) void k_grad_h16_wide(Points pts, Queries q,
                                                                 const uint16_t *__restrict__ packed, TrainArgs args,
                                                                 float *__restrict__ partials,
                                                                 float *__restrict__ loss_partials) {
    static_assert(W == 128, "wide gradient kernel");
    constexpr H16Layout L{W};
    constexpr int MT = W / 16, KB = W / 32;
    using S = Grad16WideLds<W>;
    __shared__ u32x4 smem4[(S::kTotal + 7) / 8];
    __shared__ float sLoss[kWaves16];
    uint16_t *smem = (uint16_t *)smem4;
    // sweep 0 rows: h1..h3 at 0..3W, delta2..delta4 at 3W..6W
    // sweep 1 rows: h4 at 0, delta1 at W, features at 2W, d5 at 2W + 160
    uint16_t *rH = smem;
    uint16_t *rD = smem + (SWEEP == 0 ? 3 : 1) * W * kRow16;
    uint16_t *rE = smem + 2 * W * kRow16;
    uint16_t *rD5 = rE + kFeat * kRow16;

    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, col = lane & 15, g = lane >> 4;
    const int64_t B = q.count;
    const bool use_loss = args.target != nullptr;
    const float ls = args.dyn_scale ? *args.dyn_scale * (float)B : args.loss_scale;
    const float kscale = use_loss ? 2.0f * ls / (3.0f * (float)B) : ls;

    constexpr int NACC = SWEEP == 0 ? 3 * 2 * MT : 3 * MT + 2;
    f32x4 acc[NACC];
#pragma unroll
    for (int i = 0; i < NACC; ++i) acc[i] = f32x4{0.f, 0.f, 0.f, 0.f};
    float loss_acc = 0.0f;

    const int64_t n_chunks = (B + kChunk16 - 1) / kChunk16;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        {
            const uint16_t *pk = opaque(packed);
            const int s = 16 * wave + col;
            const int64_t b = chunk * kChunk16 + s;
            const bool valid = b < B;
            const int64_t bi = valid ? b : B - 1;
            const int64_t p = query_point(q, pts, bi);
            const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};
            const float ws[3] = {q.wx[bi], q.wy[bi], q.wz[bi]};
            float f[44];
#pragma unroll
            for (int i = 0; i < 7; ++i) enc_pair2_fast(xs[i], g, f[4 * i], f[4 * i + 1], f[4 * i + 2], f[4 * i + 3]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                enc_pair2_fast(ws[i], g, f[28 + 4 * i], f[29 + 4 * i], f[30 + 4 * i], f[31 + 4 * i]);
            if constexpr (SWEEP == 1) {
#pragma unroll
                for (int t = 0; t < 28; ++t)
                    rE[feature_of(true, g, t) * kRow16 + s] = to16<PREC>((t & 1) ? 0.5f * f[t] : f[t]);
#pragma unroll
                for (int t = 0; t < 12; ++t)
                    rE[feature_of(false, g, t) * kRow16 + s] = to16<PREC>((t & 1) ? 0.5f * f[28 + t] : f[28 + t]);
            }

            u32x4 hb[4][KB];
            {
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                const uint16_t *gS = pk + L.offset(SEC_S);
#pragma unroll
                for (int kb = 0; kb < 4; ++kb) {
                    const float *fk = f + 8 * kb;
                    const u32x4 bop = kb < 3 ? u32x4{pack2<PREC>(fk[0], fk[1]), pack2<PREC>(fk[2], fk[3]),
                                                     pack2<PREC>(fk[4], fk[5]), pack2<PREC>(fk[6], fk[7])}
                                             : u32x4{pack2<PREC>(fk[0], fk[1]), pack2<PREC>(fk[2], fk[3]), 0u, 0u};
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        h[mt] = mfma16<PREC>(*(const u32x4 *)(gS + ((mt * 4 + kb) * 64 + lane) * 8), bop, h[mt]);
                }
                const float *fd = f + 28;
                const u32x4 bd0 = {pack2<PREC>(fd[0], fd[1]), pack2<PREC>(fd[2], fd[3]), pack2<PREC>(fd[4], fd[5]),
                                   pack2<PREC>(fd[6], fd[7])};
                const u32x4 bd1 = {pack2<PREC>(fd[8], fd[9]), pack2<PREC>(fd[10], fd[11]), 0u, 0u};
                const uint16_t *gD = pk + L.offset(SEC_D);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    h[mt] = mfma16<PREC>(*(const u32x4 *)(gD + ((mt * 2 + 0) * 64 + lane) * 8), bd0, h[mt]);
                    h[mt] = mfma16<PREC>(*(const u32x4 *)(gD + ((mt * 2 + 1) * 64 + lane) * 8), bd1, h[mt]);
                }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[0][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const uint16_t *sec = pk + L.offset(SEC_H0 + (l - 1));
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        h[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), hb[l - 1][kb],
                                             h[mt]);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[l][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const uint16_t *sec = pk + L.offset(SEC_O);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    z5 = mfma16<PREC>(*(const u32x4 *)(sec + (kb * 64 + lane) * 8), hb[3][kb], z5);
            }
            if constexpr (SWEEP == 0) {
#pragma unroll
                for (int l = 0; l < 3; ++l) stage_chain<W>(rH + l * W * kRow16, hb[l], g, s);
            } else {
                stage_chain<W>(rH, hb[3], g, s);
            }

            float d5[3] = {0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const float t = use_loss ? args.target[3 * b + c] : 0.0f;
                    const float dr = use_loss ? 0.0f : args.d_rgb[3 * b + c];
                    float lt;
                    d5[c] = out_grad16(z5[c], t, dr, use_loss, args.loss_eps, kscale, args.loss_kind == NIRC_LOSS_REL_L2,
                                       args.fr ? args.fr[c] : 0.0f, args.sig != 0, lt);
                    loss_acc += lt;
                }
            }
            if constexpr (SWEEP == 1) {
                if (g == 0) {
#pragma unroll
                    for (int c = 0; c < 4; ++c) rD5[c * kRow16 + s] = to16<PREC>(c < 3 ? d5[c] : 0.0f);
                }
            }

            f32x4 dl[MT];
            {
                const u32x4 bop = g == 0 ? u32x4{pack2<PREC>(d5[0], d5[1]), pack2<PREC>(d5[2], 0.0f), 0u, 0u}
                                         : u32x4{0u, 0u, 0u, 0u};
                const uint16_t *sec = pk + L.offset(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + (mt * 64 + lane) * 8), bop, f32x4{0.f, 0.f, 0.f, 0.f});
            }
#pragma unroll
            for (int l = 3; l >= 0; --l) {
                u32x4 db[KB];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint16_t hv = half_of(hb[l][mt >> 1], 4 * (mt & 1) + i);
                        if (hv == 0) dl[mt][i] = 0.0f;
                    }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) db[kb] = chain_plain<PREC>(dl[2 * kb], dl[2 * kb + 1]);
                // delta_{l+1}: sweep 0 keeps delta2..delta4 (l = 1..3), sweep 1 keeps delta1 (l = 0)
                if constexpr (SWEEP == 0) {
                    if (l >= 1) stage_chain<W>(rD + (l - 1) * W * kRow16, db, g, s);
                } else {
                    if (l == 0) stage_chain<W>(rD, db, g, s);
                }
                if (l == 0) break;
                const uint16_t *sec = pk + L.offset(SEC_T0 + (l - 1));
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) dl[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), db[kb], dl[mt]);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kb = 0; kb < kChunk16 / 32; ++kb) {
            const int s0 = 32 * kb + 8 * g;
            if constexpr (SWEEP == 0) {
                // W_{a+2} = delta_{a+2} h_{a+1}^T: A rows of delta (rD slot a), B rows of h (rH slot a)
#pragma unroll
                for (int a = 0; a < 3; ++a)
#pragma unroll
                    for (int cc = 0; cc < 2; ++cc) {
                        const int ct = 2 * wave + cc;
                        const u32x4 bv = *(const u32x4 *)(rH + (a * W + 16 * ct + col) * kRow16 + s0);
#pragma unroll
                        for (int mt = 0; mt < MT; ++mt) {
                            const u32x4 av = *(const u32x4 *)(rD + (a * W + 16 * mt + col) * kRow16 + s0);
                            acc[(a * 2 + cc) * MT + mt] = mfma16<PREC>(av, bv, acc[(a * 2 + cc) * MT + mt]);
                        }
                    }
            } else {
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const int input = wave + 4 * a;
                    if (input >= kInputs) break;
                    const u32x4 bv = *(const u32x4 *)(rE + (16 * input + col) * kRow16 + s0);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        const u32x4 av = *(const u32x4 *)(rD + (16 * mt + col) * kRow16 + s0);
                        acc[a * MT + mt] = mfma16<PREC>(av, bv, acc[a * MT + mt]);
                    }
                }
                u32x4 av5 = u32x4{0u, 0u, 0u, 0u};
                if (col < 3) av5 = *(const u32x4 *)(rD5 + col * kRow16 + s0);
#pragma unroll
                for (int cc = 0; cc < 2; ++cc) {
                    const u32x4 bv = *(const u32x4 *)(rH + (16 * (2 * wave + cc) + col) * kRow16 + s0);
                    acc[3 * MT + cc] = mfma16<PREC>(av5, bv, acc[3 * MT + cc]);
                }
            }
        }
        __syncthreads();
    }

    float *out = partials + (int64_t)blockIdx.x * n_params(W);
    if constexpr (SWEEP == 0) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        out[w_offset(W, 1 + a) + (int64_t)(16 * mt + 4 * g + i) * W + 16 * (2 * wave + cc) + col] =
                            acc[(a * 2 + cc) * MT + mt][i];
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
        if (g == 0) {
#pragma unroll
            for (int cc = 0; cc < 2; ++cc)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    out[w_offset(W, 4) + (int64_t)i * W + 16 * (2 * wave + cc) + col] = acc[3 * MT + cc][i];
        }
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) loss_acc += __shfl_xor(loss_acc, d, 64);
        if (lane == 0) sLoss[wave] = loss_acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            float t = 0.0f;
            for (int w = 0; w < kWaves16; ++w) t += sLoss[w];
            loss_partials[blockIdx.x] = t;
        }
    }
}

int train_blocks16(int64_t batch) {
    int64_t chunks = (batch + kChunk16 - 1) / kChunk16;
    if (chunks > kMaxResidentBlocks) chunks = kMaxResidentBlocks;
    return (int)(chunks < 1 ? 1 : chunks);
}

hipError_t launch_grad_partials16(int W, int prec, const Points &pts, const Queries &q, const void *packed,
                                  TrainArgs a, float *partials, float *loss_partials, int nblocks, hipStream_t s) {
    const uint16_t *pk = (const uint16_t *)packed;
    if (W == 128) {
        const dim3 grid(nblocks), block(kWaves16 * 64);
        if (prec == NIRC_BF16) {
            hipLaunchKernelGGL((k_grad_h16_wide<128, NIRC_BF16, 0>), grid, block, 0, s, pts, q, pk, a, partials,
                               loss_partials);
            hipLaunchKernelGGL((k_grad_h16_wide<128, NIRC_BF16, 1>), grid, block, 0, s, pts, q, pk, a, partials,
                               loss_partials);
        } else {
            hipLaunchKernelGGL((k_grad_h16_wide<128, NIRC_FP16, 0>), grid, block, 0, s, pts, q, pk, a, partials,
                               loss_partials);
            hipLaunchKernelGGL((k_grad_h16_wide<128, NIRC_FP16, 1>), grid, block, 0, s, pts, q, pk, a, partials,
                               loss_partials);
        }
        return hipGetLastError();
    }
    if (W != 64) return hipErrorInvalidValue;
    const bool plain = a.target && a.loss_kind == NIRC_LOSS_REL_L2 && !a.fr && !a.sig;
    if (prec == NIRC_BF16 && plain)
        hipLaunchKernelGGL((k_grad_h16<64, NIRC_BF16, true>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, pk, a,
                           partials, loss_partials);
    else if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_grad_h16<64, NIRC_BF16>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, pk, a,
                           partials, loss_partials);
    else if (plain)
        hipLaunchKernelGGL((k_grad_h16<64, NIRC_FP16, true>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, pk, a,
                           partials, loss_partials);
    else
        hipLaunchKernelGGL((k_grad_h16<64, NIRC_FP16>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, pk, a,
                           partials, loss_partials);
    return hipGetLastError();
}

hipError_t launch_train_step_multi(const TrainDesc *desc, int prec, uint32_t step, int64_t max_batch, hipStream_t s) {
    hipError_t e = launch_train_batch_multi(desc, step, max_batch, s);
    if (e != hipSuccess) return e;
    if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_grad_h16_multi<64, NIRC_BF16>), dim3(kMaxResidentBlocks), dim3(kWaves16 * 64), 0, s, desc);
    else
        hipLaunchKernelGGL((k_grad_h16_multi<64, NIRC_FP16>), dim3(kMaxResidentBlocks), dim3(kWaves16 * 64), 0, s, desc);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_reduce_grad_multi(desc, 64, s);
    if (e == hipSuccess) e = launch_adam_pack16_multi(desc, 64, prec, s);
    return e;
}

// ------------------------------------------------------------------------------------------
// The hash-grid model (width 64): the same two phases as k_grad_h16 with the 64 grid / SH / phi
// inputs.  In addition, after the first layer's delta, each sample's gradient with respect to
// its 24 grid values (W1_grid^T delta1, from the TS section) is scattered into the grid-entry
// gradient: each of the 8 corners of the sample's cell at a level receives its trilinear weight
// times the level's two values, by 64-bit fixed-point integer atomic adds (grid_acc_add; zero
// values are skipped), so that the sums do not depend on the order of the adds.
namespace {
constexpr int kScatRow = 28;   // per sample: 24 grid-value gradients, position, pad
struct HashGrad16Lds {
    static constexpr int kH = 4 * 64 * kRow16;
    static constexpr int kD = 4 * 64 * kRow16;
    static constexpr int kD5 = 4 * kRow16;
    static constexpr int kE = kHashIn * kRow16;
    static constexpr int kTotal = kH + kD + kD5 + kE;
};
}  // namespace

template <int PREC>
__global__ __launch_bounds__(kWaves16 * 64) void k_hash_grad_h16(Points pts, Queries q,
                                                                 const uint16_t *__restrict__ packed,
                                                                 const float2 *__restrict__ table, HashGridArgs grid,
                                                                 TrainArgs args, float *__restrict__ partials,
                                                                 float *__restrict__ loss_partials,
                                                                 GridAcc gacc) {
    constexpr int MT = 4, KB = 2, W = 64;
    using S = HashGrad16Lds;
    __shared__ u32x4 smem4[(S::kTotal + 7) / 8];
    __shared__ float sLoss[kWaves16];
    __shared__ HashLevel s_lv[kHashLevels];
    __shared__ float sScat[kWaves16 * 16 * kScatRow];
    uint16_t *smem = (uint16_t *)smem4;
    uint16_t *sH = smem;
    uint16_t *sD = sH + S::kH;
    uint16_t *sD5 = sD + S::kD;
    uint16_t *sE = sD5 + S::kD5;
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

    const int64_t n_chunks = (B + kChunk16 - 1) / kChunk16;
    for (int64_t chunk = blockIdx.x; chunk < n_chunks; chunk += gridDim.x) {
        {
            const uint16_t *pk = opaque(packed);
            const int s = 16 * wave + col;
            const int64_t b = chunk * kChunk16 + s;
            const bool valid = b < B;
            const int64_t bi = valid ? b : B - 1;
            const int64_t p = query_point(q, pts, bi);
            const float xs[7] = {pts.px[p], pts.py[p], pts.pz[p], pts.nx[p], pts.ny[p], pts.nz[p], pts.rough[p]};

            // inputs: operands for the MFMAs and 16-bit rows [canonical input][sample] for dW1
            u32x4 b0, b1;
            float v[6], ph[15];
            hash_surface_operands<PREC>(s_lv, grid.tmask, table, xs, g, b0, b1, v, ph);
            float Y[25];
            sh25(q.wx[bi], q.wy[bi], q.wz[bi], Y);
            const u32x4 bd0 = sh_operand_of<PREC>(Y, g);
            // the rows hold exactly the 16-bit operand values
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                sE[hash_surface_input(0, g, j) * kRow16 + s] = half_of(b0, j);
                if (8 * g + j < 25) sE[(24 + 8 * g + j) * kRow16 + s] = half_of(bd0, j);
            }
            if (g == 0) {
#pragma unroll
                for (int j = 0; j < 7; ++j) sE[(57 + j) * kRow16 + s] = half_of(b1, j);
            }

            // forward
            u32x4 hb[4][KB];
            {
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
                hash_layer1_surface<PREC>(h, pk + kHashSecS, b0, b1, lane);
                const uint16_t *gD = pk + kHashSecD;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = mfma16<PREC>(*(const u32x4 *)(gD + (mt * 64 + lane) * 8), bd0, h[mt]);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[0][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
#pragma unroll
            for (int l = 1; l < 4; ++l) {
                const uint16_t *sec = pk + hash_sec(SEC_H0 + (l - 1));
                f32x4 h[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) h[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        h[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), hb[l - 1][kb],
                                             h[mt]);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) hb[l][kb] = chain_operand<PREC>(h[2 * kb], h[2 * kb + 1]);
            }
            f32x4 z5 = f32x4{0.f, 0.f, 0.f, 0.f};
            {
                const uint16_t *sec = pk + hash_sec(SEC_O);
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) z5 = mfma16<PREC>(*(const u32x4 *)(sec + (kb * 64 + lane) * 8), hb[3][kb], z5);
            }
#pragma unroll
            for (int l = 0; l < 4; ++l) stage_chain<W>(sH + l * W * kRow16, hb[l], g, s);

            float d5[3] = {0.f, 0.f, 0.f};
            if (g == 0 && valid) {
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    float lt;
                    d5[c] = out_grad16(z5[c], args.target[3 * b + c], 0.0f, true, args.loss_eps, kscale, rel, 0.0f,
                                       false, lt);
                    loss_acc += lt;
                }
            }
            if (g == 0) {
#pragma unroll
                for (int c = 0; c < 4; ++c) sD5[c * kRow16 + s] = to16<PREC>(c < 3 ? d5[c] : 0.0f);
            }

            // backward
            f32x4 dl[MT];
            u32x4 db1[KB];   // delta1 as chained B operands
            {
                const u32x4 bop = g == 0 ? u32x4{pack2<PREC>(d5[0], d5[1]), pack2<PREC>(d5[2], 0.0f), 0u, 0u}
                                         : u32x4{0u, 0u, 0u, 0u};
                const uint16_t *sec = pk + hash_sec(SEC_OT);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
                    dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + (mt * 64 + lane) * 8), bop, f32x4{0.f, 0.f, 0.f, 0.f});
            }
#pragma unroll
            for (int l = 3; l >= 0; --l) {
                u32x4 db[KB];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const uint16_t hv = half_of(hb[l][mt >> 1], 4 * (mt & 1) + i);
                        if (hv == 0) dl[mt][i] = 0.0f;
                    }
#pragma unroll
                for (int kb = 0; kb < KB; ++kb) db[kb] = chain_plain<PREC>(dl[2 * kb], dl[2 * kb + 1]);
                stage_chain<W>(sD + l * W * kRow16, db, g, s);
                if (l == 0) {
                    db1[0] = db[0];
                    db1[1] = db[1];
                    break;
                }
                const uint16_t *sec = pk + hash_sec(SEC_T0 + (l - 1));
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) dl[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt)
                        dl[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), db[kb], dl[mt]);
            }
            // gradient of the grid values: rows 16 mt + 4 g + i of W1_grid^T delta1 for this
            // sample (column col); rows 2 k and 2 k + 1 are the two values of level k
            const uint16_t *sec = pk + kHashSecTS;
            f32x4 de[2];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                de[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int kb = 0; kb < KB; ++kb)
                    de[mt] = mfma16<PREC>(*(const u32x4 *)(sec + ((mt * KB + kb) * 64 + lane) * 8), db1[kb],
                                          de[mt]);
            }
            // scatter.  The L2 performs float atomics per cache line and instruction, so the 16
            // values of one (sample, level) - 8 corners x 2 features - go to 16 consecutive lanes,
            // corners along x (neighbouring entries: dense rows, and the hash's x multiplier is 1)
            // in consecutive lane pairs; one instruction covers 4 (sample, level) pairs.  The
            // wave's gradients and positions are staged in LDS first.
            float *sg = sScat + wave * (16 * kScatRow);
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int k = 16 * mt + 4 * g + i;
                    if (k < 24) sg[col * kScatRow + k] = valid ? de[mt][i] : 0.0f;
                }
            if (g == 0) {
                sg[col * kScatRow + 24] = xs[0];
                sg[col * kScatRow + 25] = xs[1];
                sg[col * kScatRow + 26] = xs[2];
            }
            wave_sync();
            {
                const int q = lane >> 4, corner = (lane & 15) >> 1, f = lane & 1;
#pragma unroll 4
                for (int it = 0; it < 16 * kHashLevels / 4; ++it) {
                    const int pr = 4 * it + q;
                    const int smp = pr / kHashLevels, level = pr - kHashLevels * smp;
                    const float *row = sg + smp * kScatRow;
                    const float d = row[2 * level + f];
                    const HashLevel lv = s_lv[level];
                    const HashCell cell = hash_cell(row[24], row[25], row[26], lv.res);
                    float w;
                    const uint32_t e = hash_entry(lv, grid.tmask, cell, corner, w);
                    grid_acc_add(gacc, 2 * (size_t)e + f, w * d);
                }
            }
        }
        __syncthreads();
        // phase 2: owned weight-gradient tiles (W1: inputs 16 wave .. 16 wave + 15)
#pragma unroll
        for (int kb = 0; kb < kChunk16 / 32; ++kb) {
            const int s0 = 32 * kb + 8 * g;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const u32x4 bv = *(const u32x4 *)(sH + (a * W + 16 * wave + col) * kRow16 + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const u32x4 av = *(const u32x4 *)(sD + ((a + 1) * W + 16 * mt + col) * kRow16 + s0);
                    gh[a][mt] = mfma16<PREC>(av, bv, gh[a][mt]);
                }
            }
            {
                const u32x4 bv = *(const u32x4 *)(sH + (3 * W + 16 * wave + col) * kRow16 + s0);
                u32x4 av = u32x4{0u, 0u, 0u, 0u};
                if (col < 3) av = *(const u32x4 *)(sD5 + col * kRow16 + s0);
                g5 = mfma16<PREC>(av, bv, g5);
            }
            {
                const u32x4 bv = *(const u32x4 *)(sE + (16 * wave + col) * kRow16 + s0);
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const u32x4 av = *(const u32x4 *)(sD + (16 * mt + col) * kRow16 + s0);
                    g1[mt] = mfma16<PREC>(av, bv, g1[mt]);
                }
            }
        }
        __syncthreads();
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
        for (int w = 0; w < kWaves16; ++w) t += sLoss[w];
        loss_partials[blockIdx.x] = t;
    }
}

hipError_t launch_hash_grad(int prec, const Points &pts, const Queries &q, const uint16_t *packed, const float *table,
                            const HashGridArgs &grid, TrainArgs a, float *partials, float *loss_partials,
                            GridAcc gacc, int nblocks, hipStream_t s) {
    if (!a.target) return hipErrorInvalidValue;
    const float2 *t2 = (const float2 *)table;
    if (prec == NIRC_BF16)
        hipLaunchKernelGGL((k_hash_grad_h16<NIRC_BF16>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, packed, t2,
                           grid, a, partials, loss_partials, gacc);
    else if (prec == NIRC_FP16)
        hipLaunchKernelGGL((k_hash_grad_h16<NIRC_FP16>), dim3(nblocks), dim3(kWaves16 * 64), 0, s, pts, q, packed, t2,
                           grid, a, partials, loss_partials, gacc);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace nirc
