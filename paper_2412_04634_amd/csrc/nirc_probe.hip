// Microbenchmarks behind the measured peaks: the rate a kernel of independent MFMA chains reaches
// on this device in each precision, optionally with independent FP32 FMAs in the same waves
// (whether VALU work hides under the MFMAs); and the rate of 64-bit integer atomic adds (the
// hash-grid model's fixed-point gradient scatter) by how many lanes of a wave share a cache line.
#include "nirc_h16.hpp"

namespace nirc {
namespace {

constexpr int kProbeChains = 8;   // independent accumulators per wave
constexpr int kProbeUnroll = 32;  // iterations per loop trip

template <int PREC, int FMAS>
__global__ __launch_bounds__(256) void k_probe_mfma(int iters, float *__restrict__ sink) {
    const int lane = threadIdx.x & 63;
    f32x4 acc[kProbeChains];
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) acc[c] = f32x4{0.f, 0.f, 0.f, 0.f};
    float v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = (float)(lane + k);
    // operands of 1.0 (16-bit pairs) or small floats: the sums stay far from overflow
    const uint32_t one = PREC == NIRC_BF16 ? 0x3F803F80u : 0x3C003C00u;
    const u32x4 a = u32x4{one, one, one, one};
    const float af = 1.0f + 1e-3f * (float)lane;
    u32x4 b = a;
    float bf = af;
    // kProbeUnroll iterations per trip (iters is a multiple of it): the register allocator
    // rotates the 16-bit accumulators through copies at the loop's back edge, which a long trip
    // makes negligible
    for (int it = 0; it < iters; it += kProbeUnroll) {
        // the operands stay in VGPRs and the accumulators are pinned to AGPRs at each trip's end
        // (empty asm statements that "change" them)
        asm volatile("" : "+v"(b), "+v"(bf));
#pragma unroll
        for (int h = 0; h < kProbeUnroll; ++h) {
#pragma unroll
            for (int c = 0; c < kProbeChains; ++c) {
                if constexpr (PREC == NIRC_FP32) acc[c] = mfma4(bf, 0.5f, acc[c]);
                else acc[c] = mfma16<PREC>(b, b, acc[c]);
            }
#pragma unroll
            for (int k = 0; k < FMAS; ++k) v[k & 7] = fmaf(v[k & 7], 0.999f, 0.25f);
        }
#pragma unroll
        for (int c = 0; c < kProbeChains; ++c) asm volatile("" : "+a"(acc[c]));
    }
    float t = 0.0f;
#pragma unroll
    for (int c = 0; c < kProbeChains; ++c) t += (acc[c][0] + acc[c][1]) + (acc[c][2] + acc[c][3]);
#pragma unroll
    for (int k = 0; k < 8; ++k) t += v[k];
    sink[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = t;
}

template <int PREC>
hipError_t launch_probe(int iters, int fmas, int blocks, float *sink, hipStream_t s) {
    const dim3 grid((unsigned)blocks), block(256);
    if (fmas == 0) hipLaunchKernelGGL((k_probe_mfma<PREC, 0>), grid, block, 0, s, iters, sink);
    else if (fmas == 32) hipLaunchKernelGGL((k_probe_mfma<PREC, 32>), grid, block, 0, s, iters, sink);
    else hipLaunchKernelGGL((k_probe_mfma<PREC, 64>), grid, block, 0, s, iters, sink);
    return hipGetLastError();
}

// Thread t adds 1 to element e(i) for i = t + r * T (T threads, r < reps): lanes_per_line
// consecutive i share a 128-byte line (16 elements), consecutive groups take consecutive lines,
// wrapping at the buffer's end (its length a power of two).
__global__ __launch_bounds__(256) void k_probe_atomics(int lanes_per_line, int reps, unsigned long long *buf,
                                                       int64_t mask) {
    const int64_t T = (int64_t)gridDim.x * blockDim.x;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int r = 0; r < reps; ++r) {
        const int64_t i = t + r * T;
        const int64_t e = ((i / lanes_per_line) * 16 + i % lanes_per_line) & mask;
        atomicAdd(buf + e, 1ull);
    }
}

}  // namespace
}  // namespace nirc

extern "C" nirc_status nirc_probe_mfma(int32_t precision, int32_t iters, int32_t fmas, int32_t blocks, float *sink,
                                       void *stream) {
    using namespace nirc;
    if (iters < kProbeUnroll || iters > (1 << 24) || iters % kProbeUnroll || blocks < 1 || blocks > (1 << 16) || !sink ||
        (fmas != 0 && fmas != 32 && fmas != 64))
        return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    if (precision == NIRC_FP32) e = launch_probe<NIRC_FP32>(iters, fmas, blocks, sink, s);
    else if (precision == NIRC_BF16) e = launch_probe<NIRC_BF16>(iters, fmas, blocks, sink, s);
    else if (precision == NIRC_FP16) e = launch_probe<NIRC_FP16>(iters, fmas, blocks, sink, s);
    else return NIRC_ERR_INVALID_ARG;
    return e == hipSuccess ? NIRC_OK : NIRC_ERR_HIP;
}

extern "C" nirc_status nirc_probe_atomics(int32_t lanes_per_line, int32_t reps, int32_t blocks, uint64_t *buf,
                                          int64_t buf_elems, void *stream) {
    using namespace nirc;
    if (lanes_per_line < 1 || lanes_per_line > 16 || (lanes_per_line & (lanes_per_line - 1)) || reps < 1 ||
        reps > 4096 || blocks < 1 || blocks > (1 << 20) || !buf || buf_elems < 16 || (buf_elems & (buf_elems - 1)))
        return NIRC_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_probe_atomics, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, (int)lanes_per_line,
                       (int)reps, (unsigned long long *)buf, buf_elems - 1);
    return hipGetLastError() == hipSuccess ? NIRC_OK : NIRC_ERR_HIP;
}
