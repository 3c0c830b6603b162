// Frame statistics in FP64: the exact reflected radiance of the lobe field, the mean relative
// squared error of an estimate against it, and per-point sums over seeds (unbiasedness).
//
// Ground truth with f_r = 1/pi and p = cos/pi: F(x, n) = sum_j a_j(x) J(kappa_j, mu_j . n) with
//   J(kappa, t) = (1/pi) int_{H+(n)} exp(kappa (mu . w - 1)) (n . w) dw
//               = 2 e^{-kappa} int_0^1 u e^{kappa t u} I0(kappa sqrt(1-t^2) sqrt(1-u^2)) du
// (rotate n to +z and integrate the azimuth, which yields 2 pi I0).  J is entire in t, so a
// Chebyshev expansion in t converges super-geometrically; each lobe's expansion is built once
// per set of kappas (it does not depend on the lobe axis, so a rotating scene reuses it).
#include "nirc_kernels.hpp"

namespace nirc {

namespace {

constexpr int kGL = 128;   // Gauss-Legendre nodes for J
// Chebyshev coefficients per lobe: TLMC_CHEB_COEFFS (nirc.h)

__device__ double bessel_i0(double z) {
    const double q = 0.25 * z * z;
    double term = 1.0, sum = 1.0;
    for (int k = 1; k < 400; ++k) {
        term *= q / ((double)k * (double)k);
        const double ns = sum + term;
        if (ns == sum) break;
        sum = ns;
    }
    return sum;
}

// Node i of the kGL-point Gauss-Legendre rule on [-1, 1] by Newton iteration on P_n.
__device__ void gl_node(int i, double &x, double &w) {
    const int n = kGL;
    double t = cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 60; ++it) {
        double p0 = 1.0, p1 = t;
        for (int k = 2; k <= n; ++k) {
            const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (t * p1 - p0) / (t * t - 1.0);
        const double dt = p1 / dp;
        t -= dt;
        if (fabs(dt) < 1e-15) break;
    }
    double p0 = 1.0, p1 = t;
    for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
    }
    dp = n * (t * p1 - p0) / (t * t - 1.0);
    x = t;
    w = 2.0 / ((1.0 - t * t) * dp * dp);
}

}  // namespace

// One workgroup per lobe: GL nodes into LDS, J at the Chebyshev nodes, then the coefficients
//   c_k = (2/M) sum_m J(t_m) cos(pi k (m + 1/2) / M),  t_m = cos(pi (m + 1/2) / M),
// with c_0 halved so that J(t) = sum_k c_k T_k(t).
__global__ __launch_bounds__(256) void k_reference_table(nirc_lobes lobes, double *table) {
    constexpr int M = TLMC_CHEB_COEFFS;
    __shared__ double sx[kGL], sw[kGL], sJ[M];
    const int j = blockIdx.x;
    const double kappa = lobes.kappa[j];
    for (int i = threadIdx.x; i < kGL; i += blockDim.x) gl_node(i, sx[i], sw[i]);
    __syncthreads();
    for (int m = threadIdx.x; m < M; m += blockDim.x) {
        const double t = cos(M_PI * (m + 0.5) / M);
        const double s = sqrt(fmax(0.0, 1.0 - t * t));
        double acc = 0.0;
        for (int i = 0; i < kGL; ++i) {
            const double u = 0.5 * (sx[i] + 1.0);   // map [-1,1] -> [0,1]
            acc += 0.5 * sw[i] * u * exp(kappa * (t * u - 1.0)) * bessel_i0(kappa * s * sqrt(1.0 - u * u));
        }
        sJ[m] = 2.0 * acc;
    }
    __syncthreads();
    __shared__ double sc[M];
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double c = 0.0;
        for (int m = 0; m < M; ++m) c += sJ[m] * cos(M_PI * k * (m + 0.5) / M);
        c *= 2.0 / M;
        if (k == 0) c *= 0.5;
        sc[k] = c;
    }
    __syncthreads();
    // coefficients below 1e-17 of the series' absolute sum do not change an FP64 result: store
    // them as exact zeros so that evaluation can stop at the last nonzero one
    if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < M; ++k) tot += fabs(sc[k]);
        int last = M - 1;
        while (last > 0 && fabs(sc[last]) <= 1e-17 * tot) --last;
        for (int k = last + 1; k < M; ++k) sc[k] = 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < M; k += blockDim.x) table[j * M + k] = sc[k];
}

// The table staged in LDS with the four lobes' coefficients of one degree side by side
// (tab[4 k + j] = c_jk), so that a degree's four coefficients are two 16-byte reads, and the
// number of leading coefficients that can be nonzero (the maximum over the four lobes; thread 0
// finds it).  Ends with a barrier.
__device__ inline int stage_cheb_table(const double *table, double *tab, int *s_nk) {
    for (int i = threadIdx.x; i < 4 * TLMC_CHEB_COEFFS; i += blockDim.x)
        tab[4 * (i % TLMC_CHEB_COEFFS) + i / TLMC_CHEB_COEFFS] = table[i];
    __syncthreads();
    if (threadIdx.x == 0) {
        int n = 1;
        for (int k = TLMC_CHEB_COEFFS - 1; k >= 1 && n == 1; --k)
            for (int j = 0; j < 4; ++j)
                if (tab[4 * k + j] != 0.0) n = k + 1;
        *s_nk = n;
    }
    __syncthreads();
    return *s_nk;
}

// J_j(t_ij) for the four lobes at NP points: Clenshaw recurrences for sum_k c_jk T_k(t_ij), run
// side by side (each degree's coefficients read once for all NP points).
template <int NP>
__device__ inline void cheb_eval(const double *tab, int nk, const double (&t)[NP][4], double (&J)[NP][4]) {
    double b1[NP][4], b2[NP][4];
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) b1[i][j] = b2[i][j] = 0.0;
    for (int k = nk - 1; k >= 1; --k) {
        const double2 c01 = *(const double2 *)(tab + 4 * k), c23 = *(const double2 *)(tab + 4 * k + 2);
        const double c[4] = {c01.x, c01.y, c23.x, c23.y};
#pragma unroll
        for (int i = 0; i < NP; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const double b0 = 2.0 * t[i][j] * b1[i][j] - b2[i][j] + c[j];
                b2[i][j] = b1[i][j];
                b1[i][j] = b0;
            }
    }
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) J[i][j] = t[i][j] * b1[i][j] - b2[i][j] + tab[j];
}

// The closed form F at NP points (indices p[i]).
template <int NP>
__device__ inline void reference_at(const nirc_lobes &L, const double *tab, int nk, const Points &pts,
                                    const int64_t (&p)[NP], double (&F)[NP][3]) {
    double t[NP][4], J[NP][4];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double n0 = pts.nx[p[i]], n1 = pts.ny[p[i]], n2 = pts.nz[p[i]];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const double d = (double)L.axis[j][0] * n0 + (double)L.axis[j][1] * n1 + (double)L.axis[j][2] * n2;
            t[i][j] = fmin(1.0, fmax(-1.0, d));
        }
    }
    cheb_eval<NP>(tab, nk, t, J);
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        const double x0 = pts.px[p[i]], x1 = pts.py[p[i]], x2 = pts.pz[p[i]];
        F[i][0] = F[i][1] = F[i][2] = 0.0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double a = (double)L.alpha[j][c] + (double)L.beta[j][c][0] * x0 +
                                 (double)L.beta[j][c][1] * x1 + (double)L.beta[j][c][2] * x2;
                F[i][c] += a * J[i][j];
            }
    }
}

__global__ void k_reference(Points pts, nirc_lobes lobes, const double *table, double *F) {
    __shared__ __align__(16) double tab[4 * TLMC_CHEB_COEFFS];
    __shared__ int s_nk;
    const int nk = stage_cheb_table(table, tab, &s_nk);
    const int64_t p[1] = {(int64_t)blockIdx.x * blockDim.x + threadIdx.x};
    if (p[0] >= pts.count) return;
    double f[1][3];
    reference_at<1>(lobes, tab, nk, pts, p, f);
    F[3 * p[0] + 0] = f[0][0];
    F[3 * p[0] + 1] = f[0][1];
    F[3 * p[0] + 2] = f[0][2];
}

constexpr int kStatBlocks = 2048;   // multiple of 64
static_assert(kStatBlocks % 64 == 0, "final reduction splits the blocks into 64 chunks");
constexpr int kStatThreads = 256;
constexpr int kStatPts = 2;   // points per thread evaluated together (3 and 4 measured slower)

// Per-block FP64 partial sums over points and channels:
//   0: (F_tl - F)^2 / (F^2 + eps)      1: (F_c - F)^2 / (F^2 + eps)   (when F_c is given)
//   2: F_r^2 / (F^2 + eps)             (when F_r is given)            3: number of terms
__global__ __launch_bounds__(kStatThreads) void k_frame_stats(Points pts, nirc_lobes lobes, const double *table,
                                                              const float *tl, const float *fc, const float *fr,
                                                              double eps, double *partials) {
    __shared__ __align__(16) double tab[4 * TLMC_CHEB_COEFFS];
    __shared__ double red[kStatThreads / 64][4];
    __shared__ int s_nk;
    const int nk = stage_cheb_table(table, tab, &s_nk);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    // this thread's points p0, p0 + S, p0 + 2 S, ... (S the grid's thread count), kStatPts at a
    // time so that each coefficient read serves all of them; they are added in that order
    const int64_t S = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p0 < pts.count; p0 += kStatPts * S) {
        int64_t p[kStatPts];
        int n = 0;
#pragma unroll
        for (int i = 0; i < kStatPts; ++i) {
            const bool in = p0 + i * S < pts.count;
            p[i] = in ? p0 + i * S : p0;
            n += in;
        }
        double F[kStatPts][3];
        reference_at<kStatPts>(lobes, tab, nk, pts, p, F);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) {
                const double inv = 1.0 / (F[i][c] * F[i][c] + eps);   // one division per channel
                const double e = (double)tl[3 * p[i] + c] - F[i][c];
                acc[0] += e * e * inv;
                if (fc) {
                    const double ec = (double)fc[3 * p[i] + c] - F[i][c];
                    acc[1] += ec * ec * inv;
                }
                if (fr) {
                    const double r = fr[3 * p[i] + c];
                    acc[2] += r * r * inv;
                }
                acc[3] += 1.0;
            }
    }
    // fixed-order reduction: wave butterflies, then waves in order
    for (int k = 0; k < 4; ++k) {
        double v = acc[k];
        for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
        acc[k] = v;
    }
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        for (int k = 0; k < 4; ++k) red[wave][k] = acc[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < kStatThreads / 64; ++w) s += red[w][threadIdx.x];
        partials[blockIdx.x * 4 + threadIdx.x] = s;
    }
}

// stats[k] = sum over blocks (fixed order: 64 contiguous chunks, then the chunk sums in order);
// stats[4] = MRSE, stats[5] = cache-level MRSE, stats[6] = relative residual second moment.
__global__ __launch_bounds__(256) void k_stats_final(const double *partials, double *stats) {
    constexpr int kChunks = 64, kPer = kStatBlocks / kChunks;
    __shared__ double part[4][kChunks];
    const int k = threadIdx.x / kChunks, c = threadIdx.x % kChunks;
    double v = 0.0;
    for (int b = c * kPer; b < (c + 1) * kPer; ++b) v += partials[b * 4 + k];
    part[k][c] = v;
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int i = 0; i < kChunks; ++i) t += part[threadIdx.x][i];
        part[threadIdx.x][0] = t;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double n = part[3][0] > 0.0 ? part[3][0] : 1.0;
        for (int i = 0; i < 4; ++i) stats[i] = part[i][0];
        stats[4] = part[0][0] / n;
        stats[5] = part[1][0] / n;
        stats[6] = part[2][0] / n;
        stats[7] = 0.0;
    }
}

__global__ void k_accumulate(const float *v, int64_t n, double *sum, double *sumsq) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = v[i];
    sum[i] += x;
    sumsq[i] += x * x;
}

// ------------------------------------------------------------------------------------------

hipError_t launch_reference_table(const nirc_lobes &lobes, double *table, hipStream_t s) {
    hipLaunchKernelGGL(k_reference_table, dim3(4), dim3(256), 0, s, lobes, table);
    return hipGetLastError();
}

hipError_t launch_reference(const Points &pts, const nirc_lobes &lobes, const double *table, double *F,
                            hipStream_t s) {
    if (pts.count == 0) return hipSuccess;
    hipLaunchKernelGGL(k_reference, dim3((unsigned)((pts.count + 255) / 256)), dim3(256), 0, s, pts, lobes, table, F);
    return hipGetLastError();
}

hipError_t launch_frame_stats(const Points &pts, const nirc_lobes &lobes, const double *table, const float *tl,
                              const float *fc, const float *fr, double eps, double *scratch, double *stats,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_frame_stats, dim3(kStatBlocks), dim3(kStatThreads), 0, s, pts, lobes, table, tl, fc, fr,
                       eps, scratch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(256), 0, s, scratch, stats);
    return hipGetLastError();
}

size_t frame_stats_scratch_bytes() { return (size_t)kStatBlocks * 4 * sizeof(double); }

hipError_t launch_accumulate(const float *v, int64_t n, double *sum, double *sumsq, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_accumulate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, v, n, sum, sumsq);
    return hipGetLastError();
}

}  // namespace nirc
