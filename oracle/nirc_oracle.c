/*
 * FP64 CPU oracle for the neural incident radiance cache (NIRC) and the two-level Monte Carlo
 * estimator.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU-baseline
 * leg call it; the HIP library never does.  It shares no code, header or table with the HIP path.
 *
 * Everything is plain loops in double precision (OpenMP only over independent points/queries),
 * written so that each step can be checked against the paper by eye:
 *
 *   - cache-level estimator   F_c = (1/N_c) sum_k f_c(X_k)/p_c(X_k)          (eq. Fc; eq. L_c)
 *   - residual estimator      F_r = (1/N_r) sum (f(Y) - f_c(Y))/p_r(Y)        (eq. Fr; eq. L_r)
 *   - two-level estimator     F_tl = F_c + F_r                                 (eq. Fml; eq. L_mlmc)
 *     With a white Lambertian BRDF (1/pi) and cosine-weighted sampling (p = cos/pi) the factor
 *     f_r cos / p is exactly 1, so F_c is the mean of the N cache predictions and F_r is the
 *     target radiance minus the cache prediction at one independent direction.
 *   - the cache is an MLP (4 hidden ReLU layers, no biases, Sec. "Results": 4 hidden layers of
 *     width 64, ReLU) on a sin/cos frequency encoding of (x, omega, n, roughness), with an
 *     exponential output so that radiance predictions stay positive.
 *   - training loss: relative L2 with a stop-gradient denominator (eq. 12), read on radiance
 *     with p_r = 1; Adam (Sec. "Results": Adam, several steps per frame).
 *   - ground truth: the cosine-weighted integral of the lobe field, reduced to a 1D integral
 *     with a modified Bessel function and evaluated with Gauss-Legendre quadrature.
 *
 * Random numbers the method draws (sampling directions, training samples) come from
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11), implemented here from its published definition.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NIN 10
#define NFREQ 8
#define NFEAT 160
#define NLOBES 4

/* ------------------------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al. SC'11): 10 rounds of the multiply-xor S-box on a 4x32 counter;
 * the two key words advance by the Weyl constants (golden ratio, sqrt(3)-1) between rounds.    */
void oracle_philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* A 24-bit uniform in [0,1) from one 32-bit word. */
static double u24(uint32_t r) { return (double)(r >> 8) * (1.0 / 16777216.0); }

/* Counter streams of the method's random numbers. */
enum { STREAM_CACHE_DIR = 3, STREAM_RESIDUAL_DIR = 4, STREAM_TRAIN = 5, STREAM_TERMINATE = 6 };

/* The two uniforms of sampled direction k of point p in frame f.  One Philox block serves two
 * directions: cache directions k and k+1 (k even) of a point share counter (p, k/2, f, 3); the
 * residual directions of points p and p+1 (p even) share counter (p/2, 0, f, 4). */
static void direction_uniforms(uint64_t seed, uint32_t p, int k, int residual, uint32_t frame,
                               double *u1, double *u2)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t out[4];
    if (residual) {
        uint32_t ctr[4] = {p >> 1, 0u, frame, STREAM_RESIDUAL_DIR};
        oracle_philox(ctr, key, out);
        if (p & 1) { *u1 = u24(out[2]); *u2 = u24(out[3]); }
        else       { *u1 = u24(out[0]); *u2 = u24(out[1]); }
    } else {
        uint32_t ctr[4] = {p, (uint32_t)(k >> 1), frame, STREAM_CACHE_DIR};
        oracle_philox(ctr, key, out);
        if (k & 1) { *u1 = u24(out[2]); *u2 = u24(out[3]); }
        else       { *u1 = u24(out[0]); *u2 = u24(out[1]); }
    }
}

/* Cosine-weighted hemisphere sample about the normal n (pdf cos(theta)/pi).  Local direction
 * (sqrt(u1) cos 2 pi u2, sqrt(u1) sin 2 pi u2, sqrt(1-u1)); world frame from the branchless
 * orthonormal basis of Duff et al. ("Building an Orthonormal Basis, Revisited", JCGT 2017).  */
static void cosine_direction(const double n[3], double u1, double u2, double w[3])
{
    double r = sqrt(u1);
    double lx = r * cos(2.0 * M_PI * u2);
    double ly = r * sin(2.0 * M_PI * u2);
    double lz = sqrt(1.0 - u1);
    double s = (n[2] >= 0.0) ? 1.0 : -1.0;
    double a = -1.0 / (s + n[2]);
    double b = n[0] * n[1] * a;
    double t[3] = {1.0 + s * n[0] * n[0] * a, s * b, -s * n[0]};
    double bb[3] = {b, s + n[1] * n[1] * a, -n[1]};
    for (int d = 0; d < 3; ++d) w[d] = lx * t[d] + ly * bb[d] + lz * n[d];
}

/* ids == NULL: point p of the array is point p of the frame; otherwise the arrays hold a subset
 * of a frame's points and ids[p] is the frame index of entry p (its Philox counter). */
void oracle_sample_dirs(int64_t P, const float *nx, const float *ny, const float *nz, const int64_t *ids,
                        int n_cache, uint64_t seed, uint64_t frame, double *dirs /* [P][n_cache+1][3] */)
{
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double n[3] = {nx[p], ny[p], nz[p]};
        const uint32_t id = (uint32_t)(ids ? ids[p] : p);
        for (int k = 0; k <= n_cache; ++k) {
            double u1, u2;
            direction_uniforms(seed, id, k, k == n_cache, (uint32_t)frame, &u1, &u2);
            cosine_direction(n, u1, u2, dirs + ((size_t)p * (n_cache + 1) + k) * 3);
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Frequency encoding: each of the 10 inputs v gives sin(2^k pi v), cos(2^k pi v), k = 0..7;
 * feature index 16*i + 2*k + (0: sin, 1: cos); inputs in the order x, omega, n, roughness.
 * sin/cos(pi t) use an exact reduction of t to [-1/4, 1/4] plus quadrant, so multiples of 1/2
 * give exact values.                                                                          */
static void sincospi(double t, double *s, double *c)
{
    double r = remainder(t, 2.0);          /* exact, in [-1, 1] */
    double q = nearbyint(2.0 * r);         /* quadrant in {-2..2} */
    double f = r - 0.5 * q;                /* exact, in [-1/4, 1/4] */
    double sf = sin(M_PI * f), cf = cos(M_PI * f);
    switch (((int)q) & 3) {
    case 0: *s = sf;  *c = cf;  break;
    case 1: *s = cf;  *c = -sf; break;
    case 2: *s = -sf; *c = -cf; break;
    default: *s = -cf; *c = sf; break;
    }
}

static void encode_inputs(const double in[NIN], double feat[NFEAT])
{
    for (int i = 0; i < NIN; ++i)
        for (int k = 0; k < NFREQ; ++k) {
            double s, c;
            sincospi(ldexp(in[i], k), &s, &c);
            feat[16 * i + 2 * k + 0] = s;
            feat[16 * i + 2 * k + 1] = c;
        }
}

static void gather_inputs(const float *const pts[7], int64_t p, const double w[3], double in[NIN])
{
    in[0] = pts[0][p]; in[1] = pts[1][p]; in[2] = pts[2][p];
    in[3] = w[0];      in[4] = w[1];      in[5] = w[2];
    in[6] = pts[3][p]; in[7] = pts[4][p]; in[8] = pts[5][p];
    in[9] = pts[6][p];
}

void oracle_encode(int64_t Q, const float *px, const float *py, const float *pz, const float *nx,
                   const float *ny, const float *nz, const float *rough, const int32_t *point,
                   const double *dirs /* [Q][3] */, double *feat /* [Q][160] */)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double in[NIN];
        gather_inputs(pts, point ? point[q] : q, dirs + 3 * q, in);
        encode_inputs(in, feat + (size_t)q * NFEAT);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* MLP: h1 = ReLU(W1 e), h_l = ReLU(W_l h_{l-1}) (l = 2..4), z = W5 h4, y = exp(z) for the
 * radiance cache (output 0) or y = 1 / (1 + exp(-z)) for the visibility cache (output 1, Sec.
 * "Neural Visibility Cache": visibility lies in [0, 1], hence a sigmoid on the outputs).
 * Canonical parameter vector: W1 [W x 160], W2, W3, W4 [W x W], W5 [3 x W], row-major.       */
typedef struct {
    int width;
    int vis;   /* 1: sigmoid outputs (visibility cache) */
    const double *W[5];
    int rows[5], cols[5];
} net_t;

static int64_t n_params_of(int width) { return (int64_t)width * NFEAT + 3LL * width * width + 3LL * width; }

int64_t oracle_n_params(int width) { return n_params_of(width); }

/* Thread control for timing the oracle on one core and on all of them. */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static void net_setup(net_t *net, const double *w, int width)
{
    net->width = width;
    net->vis = 0;
    int rows[5] = {width, width, width, width, 3};
    int cols[5] = {NFEAT, width, width, width, width};
    size_t off = 0;
    for (int l = 0; l < 5; ++l) {
        net->W[l] = w + off;
        net->rows[l] = rows[l];
        net->cols[l] = cols[l];
        off += (size_t)rows[l] * cols[l];
    }
}

/* Forward pass keeping pre-activations z_l (l = 0..3 hidden, 4 = output) and activations. */
typedef struct {
    double h[4][256];   /* hidden activations (width <= 256) */
    double z[4][256];   /* hidden pre-activations */
    double zo[3];       /* output pre-activation */
    double y[3];        /* output */
} acts_t;

static void net_forward(const net_t *net, const double *e, acts_t *a)
{
    const double *x = e;
    for (int l = 0; l < 4; ++l) {
        for (int r = 0; r < net->rows[l]; ++r) {
            double s = 0.0;
            for (int c = 0; c < net->cols[l]; ++c) s += net->W[l][(size_t)r * net->cols[l] + c] * x[c];
            a->z[l][r] = s;
            a->h[l][r] = s > 0.0 ? s : 0.0;
        }
        x = a->h[l];
    }
    for (int r = 0; r < 3; ++r) {
        double s = 0.0;
        for (int c = 0; c < net->cols[4]; ++c) s += net->W[4][(size_t)r * net->cols[4] + c] * x[c];
        a->zo[r] = s;
        a->y[r] = net->vis ? 1.0 / (1.0 + exp(-s)) : exp(s);
    }
}

/* Cache prediction for explicit queries (point index + direction); output 1: the visibility. */
void oracle_infer(int64_t Q, const float *px, const float *py, const float *pz, const float *nx,
                  const float *ny, const float *nz, const float *rough, const int32_t *point,
                  const double *dirs /* [Q][3] */, const double *w, int width, int output,
                  double *rgb /* [Q][3] */)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    net_t net;
    net_setup(&net, w, width);
    net.vis = output == 1;
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double in[NIN], e[NFEAT];
        acts_t a;
        gather_inputs(pts, point ? point[q] : q, dirs + 3 * q, in);
        encode_inputs(in, e);
        net_forward(&net, e, &a);
        for (int c = 0; c < 3; ++c) rgb[3 * q + c] = a.y[c];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Synthetic incident radiance: L_c(x, w) = sum_j a_jc(x) exp(kappa_j (mu_j . w - 1)),
 * a_jc(x) = alpha_jc + sum_d beta_jcd x_d.  Lobe record (64 floats): axis[4][3], kappa[4],
 * alpha[4][3], beta[4][3][3].                                                                 */
typedef struct {
    double axis[NLOBES][3], kappa[NLOBES], alpha[NLOBES][3], beta[NLOBES][3][3];
} lobes_t;

static void lobes_unpack(const float *rec, lobes_t *L)
{
    int o = 0;
    for (int j = 0; j < NLOBES; ++j) for (int d = 0; d < 3; ++d) L->axis[j][d] = rec[o++];
    for (int j = 0; j < NLOBES; ++j) L->kappa[j] = rec[o++];
    for (int j = 0; j < NLOBES; ++j) for (int c = 0; c < 3; ++c) L->alpha[j][c] = rec[o++];
    for (int j = 0; j < NLOBES; ++j)
        for (int c = 0; c < 3; ++c) for (int d = 0; d < 3; ++d) L->beta[j][c][d] = rec[o++];
}

static void lobe_amplitude(const lobes_t *L, int j, const double x[3], double a[3])
{
    for (int c = 0; c < 3; ++c) {
        a[c] = L->alpha[j][c];
        for (int d = 0; d < 3; ++d) a[c] += L->beta[j][c][d] * x[d];
    }
}

static void field_eval(const lobes_t *L, const double x[3], const double w[3], double out[3])
{
    out[0] = out[1] = out[2] = 0.0;
    for (int j = 0; j < NLOBES; ++j) {
        double a[3];
        lobe_amplitude(L, j, x, a);
        double mu_w = L->axis[j][0] * w[0] + L->axis[j][1] * w[1] + L->axis[j][2] * w[2];
        double g = exp(L->kappa[j] * (mu_w - 1.0));
        for (int c = 0; c < 3; ++c) out[c] += a[c] * g;
    }
}

/* Synthetic visibility for the visibility cache (environment lighting, Sec. "Neural Visibility
 * Cache"): a soft occluder over the first lobe's direction mu_0 that blocks 90 % of it,
 *   V(x, w) = 1 - 0.9 / (1 + exp(-16 (mu_0 . w - c(x)))),   c(x) = 0.6 + 0.3 (x_0 - 0.5),
 * so the occluded cap grows and shrinks across the scene; V is in [0.1, 1] and smooth.       */
static double visibility(const lobes_t *L, const double x[3], const double w[3])
{
    const double m = L->axis[0][0] * w[0] + L->axis[0][1] * w[1] + L->axis[0][2] * w[2];
    const double c = 0.6 + 0.3 * (x[0] - 0.5);
    return 1.0 - 0.9 / (1.0 + exp(-16.0 * (m - c)));
}

void oracle_visibility(int64_t Q, const float *lobes, const float *px, const float *py, const float *pz,
                       const int32_t *point, const double *dirs, double *out)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        int64_t p = point ? point[q] : q;
        double x[3] = {px[p], py[p], pz[p]};
        out[q] = visibility(&L, x, dirs + 3 * q);
    }
}

void oracle_field(int64_t Q, const float *lobes, const float *px, const float *py, const float *pz,
                  const int32_t *point, const double *dirs, double *out)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        int64_t p = point ? point[q] : q;
        double x[3] = {px[p], py[p], pz[p]};
        field_eval(&L, x, dirs + 3 * q, out + 3 * q);
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Two-level estimator per point and channel (eq. L_c, L_r, L_mlmc with f_r cos/p = 1, L_e = 0):
 *   F_c = (1/N) sum_k y(x, w_k),   F_r = L(x, w_r) - y(x, w_r),   F_tl = F_c + F_r.
 * dirs == NULL: sample the directions here (Philox streams as above); otherwise use the given
 * [P][N+1][3] directions (the last one of each point is the residual direction).
 * plug_in != 0 replaces the network by the field itself (y := L), a special case where F_r = 0. */
void oracle_estimate(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                     const float *ny, const float *nz, const float *rough, const float *lobes,
                     const double *w, int width, int output, int n_cache, uint64_t seed, uint64_t frame,
                     const double *dirs, int plug_in, double *out_tl, double *out_c, double *out_r)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    lobes_t L;
    lobes_unpack(lobes, &L);
    net_t net;
    net_setup(&net, w, width);
    /* output 1, the visibility cache: incident radiance is the predicted visibility times the
     * known radiance, n_V(x, w) L(x, w); the residual sample is V(x, w_r) L(x, w_r) minus it.
     * output 2, a radiance cache on the same occluded scene: the residual sample is V L. */
    const int vis = output == 1, occ = output != 0;
    net.vis = vis;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        double x[3] = {px[p], py[p], pz[p]};
        double n[3] = {nx[p], ny[p], nz[p]};
        double fc[3] = {0, 0, 0}, fr[3];
        for (int k = 0; k <= n_cache; ++k) {
            double wdir[3];
            if (dirs) {
                const double *d = dirs + ((size_t)p * (n_cache + 1) + k) * 3;
                wdir[0] = d[0]; wdir[1] = d[1]; wdir[2] = d[2];
            } else {
                double u1, u2;
                direction_uniforms(seed, (uint32_t)p, k, k == n_cache, (uint32_t)frame, &u1, &u2);
                cosine_direction(n, u1, u2, wdir);
            }
            double y[3], Lw[3];
            field_eval(&L, x, wdir, Lw);
            const double V = occ ? visibility(&L, x, wdir) : 1.0;
            if (plug_in) {
                for (int c = 0; c < 3; ++c) y[c] = V * Lw[c];
            } else {
                double in[NIN], e[NFEAT];
                acts_t a;
                gather_inputs(pts, p, wdir, in);
                encode_inputs(in, e);
                net_forward(&net, e, &a);
                for (int c = 0; c < 3; ++c) y[c] = vis ? a.y[c] * Lw[c] : a.y[c];
            }
            if (k < n_cache) {
                for (int c = 0; c < 3; ++c) fc[c] += y[c];
            } else {
                for (int c = 0; c < 3; ++c) fr[c] = V * Lw[c] - y[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            double Fc = n_cache > 0 ? fc[c] / n_cache : 0.0;
            if (out_c) out_c[3 * p + c] = Fc;
            if (out_r) out_r[3 * p + c] = fr[c];
            if (out_tl) out_tl[3 * p + c] = Fc + fr[c];
        }
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Biased estimator with the Balanced Termination Heuristic at the shading point (Sec. "Path
 * Termination Heuristics", first vertex): the path's scattering direction w_s is drawn from the
 * BRDF (cosine-weighted, pdf p = cos/pi; it is the residual direction of the two-level
 * estimator, same Philox stream), the continuation probability is P_s = p / (p + N/pi) =
 * cos / (cos + N), and a uniform xi from counter (p >> 2, 0, frame, STREAM_TERMINATE), word
 * p & 3, decides: xi > P_s stops the path and shades with the N cache samples (F_c); otherwise
 * the path continues and its radiance L(x, w_s) is the estimate (f_r cos / p = 1).
 * The decision is taken exactly: with cos = sqrt(1 - u1) of the sampler and both uniforms
 * 24-bit fractions, xi = X 2^-24 and u1 = U 2^-24,
 *   xi > cos / (cos + N)  <=>  (xi N)^2 > (1 - u1) (1 - xi)^2
 *                         <=>  (X N)^2 2^24 > (2^24 - U) (2^24 - X)^2,
 * compared in 128-bit integers (no rounding anywhere).
 * rrad (nullable): the radiance found along w_s (the field otherwise).  cont[p] = 1 where the
 * path continues. */
void oracle_estimate_biased(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                            const float *ny, const float *nz, const float *rough, const float *lobes,
                            const double *w, int width, int output, int n_cache, uint64_t seed, uint64_t frame,
                            const double *rrad, double *out, int32_t *cont)
{
    double *fc = (double *)malloc(sizeof(double) * 3 * (size_t)(P > 0 ? P : 1));
    oracle_estimate(P, px, py, pz, nx, ny, nz, rough, lobes, w, width, output, n_cache, seed, frame, NULL, 0, NULL,
                    fc, NULL);
    lobes_t L;
    lobes_unpack(lobes, &L);
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < P; ++p) {
        double u1, u2, ws[3];
        const double n[3] = {nx[p], ny[p], nz[p]};
        direction_uniforms(seed, (uint32_t)p, n_cache, 1, (uint32_t)frame, &u1, &u2);
        cosine_direction(n, u1, u2, ws);
        uint32_t ctr[4] = {(uint32_t)p >> 2, 0u, (uint32_t)frame, STREAM_TERMINATE}, r[4];
        oracle_philox(ctr, key, r);
        const unsigned __int128 X = r[p & 3] >> 8, U = (uint64_t)(u1 * 16777216.0), one = (uint64_t)1 << 24;
        const int stop = X * X * (unsigned __int128)n_cache * (unsigned __int128)n_cache * one >
                         (one - U) * (one - X) * (one - X);
        if (cont) cont[p] = !stop;
        if (stop) {
            for (int c = 0; c < 3; ++c) out[3 * p + c] = fc[3 * p + c];
        } else if (rrad) {
            for (int c = 0; c < 3; ++c) out[3 * p + c] = rrad[3 * p + c];
        } else {
            const double x[3] = {px[p], py[p], pz[p]};
            field_eval(&L, x, ws, out + 3 * p);
            if (output != 0) {   /* the continued path meets the occluder */
                const double V = visibility(&L, x, ws);
                for (int c = 0; c < 3; ++c) out[3 * p + c] *= V;
            }
        }
    }
    free(fc);
}

/* ------------------------------------------------------------------------------------------ */
/* Ground truth F(x, n) = (1/pi) int_{H+(n)} L(x, w) (n . w) dw = sum_j a_j(x) J(kappa_j, mu_j . n),
 * with, after rotating n to +z and integrating the azimuth (which gives 2 pi I0),
 *   J(kappa, t) = 2 e^{-kappa} int_0^1 u e^{kappa t u} I0(kappa sqrt(1-t^2) sqrt(1-u^2)) du.
 * The integrand is entire in u, so Gauss-Legendre converges geometrically.                    */
double oracle_bessel_i0(double z)
{
    /* power series sum_k (z^2/4)^k / (k!)^2, summed until the terms stop changing the sum */
    double q = 0.25 * z * z, term = 1.0, sum = 1.0;
    for (int k = 1; k < 500; ++k) {
        term *= q / ((double)k * (double)k);
        double ns = sum + term;
        if (ns == sum) break;
        sum = ns;
    }
    return sum;
}

/* Gauss-Legendre nodes and weights on [0, 1] (Newton iteration on P_n). */
void oracle_gauss_legendre(int n, double *x, double *wgt)
{
    for (int i = 0; i < n; ++i) {
        double t = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        {   /* derivative at the converged node */
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1; p1 = p2;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
        }
        x[i] = 0.5 * (1.0 - t);
        wgt[i] = 1.0 / ((1.0 - t * t) * dp * dp);   /* 2/((1-t^2) P'^2) mapped to [0,1] */
    }
}

static double J_on_nodes(double kappa, double t, int n, const double *xs, const double *ws)
{
    if (t > 1.0) t = 1.0;
    if (t < -1.0) t = -1.0;
    double s = sqrt(1.0 - t * t), acc = 0.0;
    for (int i = 0; i < n; ++i) {
        double u = xs[i];
        acc += ws[i] * u * exp(kappa * (t * u - 1.0)) * oracle_bessel_i0(kappa * s * sqrt(1.0 - u * u));
    }
    return 2.0 * acc;
}

double oracle_J(double kappa, double t, int n_nodes)
{
    double xs[1024], ws[1024];
    if (n_nodes > 1024) n_nodes = 1024;
    oracle_gauss_legendre(n_nodes, xs, ws);
    return J_on_nodes(kappa, t, n_nodes, xs, ws);
}

void oracle_closed_form(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                        const float *ny, const float *nz, const float *lobes, int n_nodes, double *F)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
    double xs[1024], ws[1024];
    if (n_nodes > 1024) n_nodes = 1024;
    oracle_gauss_legendre(n_nodes, xs, ws);
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t p = 0; p < P; ++p) {
        double x[3] = {px[p], py[p], pz[p]};
        double n[3] = {nx[p], ny[p], nz[p]};
        double acc[3] = {0, 0, 0};
        for (int j = 0; j < NLOBES; ++j) {
            double a[3];
            lobe_amplitude(&L, j, x, a);
            double t = L.axis[j][0] * n[0] + L.axis[j][1] * n[1] + L.axis[j][2] * n[2];
            double J = J_on_nodes(L.kappa[j], t, n_nodes, xs, ws);
            for (int c = 0; c < 3; ++c) acc[c] += a[c] * J;
        }
        for (int c = 0; c < 3; ++c) F[3 * p + c] = acc[c];
    }
}

/* Second moment of the field under cosine sampling, per channel:
 *   E[L^2] = (1/pi) int L(x, w)^2 (n . w) dw
 *          = sum_j sum_k a_j a_k e^{K_jk - kappa_j - kappa_k} J(K_jk, nu_jk . n),
 * because the product of two lobes is a lobe: kappa_j mu_j . w + kappa_k mu_k . w = K nu . w with
 * K = |kappa_j mu_j + kappa_k mu_k| and nu its direction (J(0, t) = 1).                         */
void oracle_second_moment(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                          const float *ny, const float *nz, const float *lobes, int n_nodes, double *M2)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
    double xs[1024], ws[1024];
    if (n_nodes > 1024) n_nodes = 1024;
    oracle_gauss_legendre(n_nodes, xs, ws);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        double x[3] = {px[p], py[p], pz[p]};
        double n[3] = {nx[p], ny[p], nz[p]};
        double acc[3] = {0, 0, 0};
        for (int j = 0; j < NLOBES; ++j)
            for (int k = 0; k < NLOBES; ++k) {
                double aj[3], ak[3], v[3];
                lobe_amplitude(&L, j, x, aj);
                lobe_amplitude(&L, k, x, ak);
                for (int d = 0; d < 3; ++d) v[d] = L.kappa[j] * L.axis[j][d] + L.kappa[k] * L.axis[k][d];
                double K = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
                double J = 1.0;
                if (K > 1e-12) J = J_on_nodes(K, (v[0] * n[0] + v[1] * n[1] + v[2] * n[2]) / K, n_nodes, xs, ws);
                double e = exp(K - L.kappa[j] - L.kappa[k]) * J;
                for (int c = 0; c < 3; ++c) acc[c] += aj[c] * ak[c] * e;
            }
        for (int c = 0; c < 3; ++c) M2[3 * p + c] = acc[c];
    }
}

/* ------------------------------------------------------------------------------------------ */
/* Training (Sec. "Radiance Cache Optimization", read on radiance with p_r = 1).  Three losses of
 * that section, per sample b and channel c with d = y - t:
 *   kind 0, relative L2 (eq. 12, the method's):  d^2 / (sg(y)^2 + eps);
 *   kind 1, squared difference (the plain L2 loss before the relative weighting):  d^2;
 *   kind 2, variance of the residual estimator (eq. for L_V):  (t - y - F_r)^2, with F_r the
 *           residual's expectation estimated per channel by the batch mean of t - y.
 * loss = (1/(3B)) sum_{b,c} of the term.  Gradients: dloss/dy = (2/(3B)) d / den for kinds 0
 * and 1 (den = y^2 + eps or 1, the denominator held constant), (2/(3B)) (y - t + F_r) for
 * kind 2 (F_r's own derivative adds nothing: the centred terms sum to zero over the batch);
 * dloss/dz = dloss/dy * y (y = exp z), then plain backpropagation through the ReLU layers
 * (ReLU'(0) = 0); only weight gradients.  frozen == 0 differentiates through the relative
 * loss's denominator as well (a control, not the method).                                    */
double oracle_loss_grad(int64_t B, const float *px, const float *py, const float *pz, const float *nx,
                        const float *ny, const float *nz, const float *rough, const int32_t *point,
                        const double *dirs, const double *target, const double *w, int width,
                        int output, double eps, int frozen, int kind, double *grad /* [n_params] or NULL */)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    net_t net;
    net_setup(&net, w, width);
    net.vis = output == 1;   /* sigmoid outputs: dy/dz = y (1 - y) */
    int64_t np = n_params_of(width);
    double loss = 0.0;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)np);
    int W = width;
    /* per-sample work is independent; accumulate per-thread and combine in a fixed order */
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    /* kind 2: the batch estimate of F_r = E[t - y] per channel, from a forward pass first */
    double fr[3] = {0.0, 0.0, 0.0};
    if (kind == 2) {
        double *part = (double *)calloc((size_t)nthreads * 3, sizeof(double));
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
#pragma omp for schedule(static)
            for (int64_t b = 0; b < B; ++b) {
                double in[NIN], e[NFEAT];
                acts_t a;
                gather_inputs(pts, point ? point[b] : b, dirs + 3 * b, in);
                encode_inputs(in, e);
                net_forward(&net, e, &a);
                for (int c = 0; c < 3; ++c) part[3 * tid + c] += target[3 * b + c] - a.y[c];
            }
        }
        for (int t = 0; t < nthreads; ++t)
            for (int c = 0; c < 3; ++c) fr[c] += part[3 * t + c];
        for (int c = 0; c < 3; ++c) fr[c] /= (double)B;
        free(part);
    }
    double *tg = grad ? (double *)calloc((size_t)nthreads * np, sizeof(double)) : NULL;
    double *tl = (double *)calloc((size_t)nthreads, sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = tg ? tg + (size_t)tid * np : NULL;
#pragma omp for schedule(static)
        for (int64_t b = 0; b < B; ++b) {
            double in[NIN], e[NFEAT];
            acts_t a;
            gather_inputs(pts, point ? point[b] : b, dirs + 3 * b, in);
            encode_inputs(in, e);
            net_forward(&net, e, &a);
            double dz[3];
            for (int c = 0; c < 3; ++c) {
                double y = a.y[c], t = target[3 * b + c];
                double d = (kind == 2) ? (y - t) + fr[c] : y - t;
                double den = (kind == 0) ? y * y + eps : 1.0;
                tl[tid] += d * d / den;
                double dy = 2.0 * d / den;
                if (!frozen && kind == 0) dy -= d * d * 2.0 * y / (den * den);
                dz[c] = dy * (net.vis ? y * (1.0 - y) : y) / (3.0 * (double)B);
            }
            if (!g) continue;
            /* output layer */
            double *gW5 = g + (size_t)W * NFEAT + 3LL * W * W;
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < W; ++j) gW5[(size_t)c * W + j] += dz[c] * a.h[3][j];
            double delta[256], prev[256];
            for (int j = 0; j < W; ++j) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += net.W[4][(size_t)c * W + j] * dz[c];
                delta[j] = a.z[3][j] > 0.0 ? s : 0.0;
            }
            /* hidden layers 4..2 (weight index l = 3..1) */
            for (int l = 3; l >= 1; --l) {
                double *gW = g + (size_t)W * NFEAT + (size_t)(l - 1) * W * W;
                for (int r = 0; r < W; ++r)
                    for (int c = 0; c < W; ++c) gW[(size_t)r * W + c] += delta[r] * a.h[l - 1][c];
                for (int c = 0; c < W; ++c) {
                    double s = 0.0;
                    for (int r = 0; r < W; ++r) s += net.W[l][(size_t)r * W + c] * delta[r];
                    prev[c] = a.z[l - 1][c] > 0.0 ? s : 0.0;
                }
                memcpy(delta, prev, sizeof(double) * W);
            }
            /* first layer */
            for (int r = 0; r < W; ++r)
                for (int c = 0; c < NFEAT; ++c) g[(size_t)r * NFEAT + c] += delta[r] * e[c];
        }
    }
    for (int t = 0; t < nthreads; ++t) loss += tl[t];
    if (grad)
        for (int t = 0; t < nthreads; ++t)
            for (int64_t i = 0; i < np; ++i) grad[i] += tg[(size_t)t * np + i];
    free(tg);
    free(tl);
    return loss / (3.0 * (double)B);
}

/* Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
 * w <- w - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), t = 1 for the first step.     */
void oracle_adam(int64_t n, double *w, double *m, double *v, const double *g, int64_t t, double lr,
                 double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        w[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* Training samples (the stand-in for the paper's separate training pass): sample b of training
 * step s in frame f draws one Philox block from counter (b, s, f, STREAM_TRAIN): word 0 picks the
 * point uniformly (floor(r0 * P / 2^32), integer arithmetic), words 1 and 2 give a fresh
 * cosine-weighted direction about that point's normal; the target is the noise-free field.    */
void oracle_train_batch(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                        const float *ny, const float *nz, const float *lobes, int64_t B, uint64_t seed,
                        uint64_t frame, uint32_t step, int output, int32_t *point, double *dirs, double *target)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < B; ++b) {
        uint32_t ctr[4] = {(uint32_t)b, step, (uint32_t)frame, STREAM_TRAIN}, r[4];
        oracle_philox(ctr, key, r);
        int64_t p = (int64_t)(((uint64_t)r[0] * (uint64_t)P) >> 32);
        point[b] = (int32_t)p;
        double n[3] = {nx[p], ny[p], nz[p]};
        cosine_direction(n, u24(r[1]), u24(r[2]), dirs + 3 * b);
        double x[3] = {px[p], py[p], pz[p]};
        field_eval(&L, x, dirs + 3 * b, target + 3 * b);
        if (output != 0) {   /* the occluded scene: the visibility cache learns V (in every
                                channel), the radiance cache V L */
            const double V = visibility(&L, x, dirs + 3 * b);
            for (int c = 0; c < 3; ++c) target[3 * b + c] = output == 1 ? V : V * target[3 * b + c];
        }
    }
}

/* Reference integral F(x) = (1/pi) int V(x, w) L(x, w) (n . w) dw (V = 1 for output 0, the
 * unoccluded scene) by tensor Gauss-Legendre quadrature over the uniforms (u1, u2) of the
 * cosine-weighted map, whose pdf cancels the cosine: F = int_[0,1]^2 V L (w(u1, u2)) du1 du2.
 * Test reference only. */
void oracle_quadrature(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                       const float *ny, const float *nz, const float *lobes, int output, int n_nodes, double *F)
{
    lobes_t L;
    lobes_unpack(lobes, &L);
    double *xs = (double *)malloc(sizeof(double) * (size_t)n_nodes), *ws = (double *)malloc(sizeof(double) * (size_t)n_nodes);
    oracle_gauss_legendre(n_nodes, xs, ws);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t p = 0; p < P; ++p) {
        const double x[3] = {px[p], py[p], pz[p]};
        const double n[3] = {nx[p], ny[p], nz[p]};
        double acc[3] = {0, 0, 0};
        for (int i = 0; i < n_nodes; ++i)
            for (int k = 0; k < n_nodes; ++k) {
                const double u1 = xs[i], u2 = xs[k], wt = ws[i] * ws[k];   /* nodes on [0, 1] */
                double wd[3], Lw[3];
                cosine_direction(n, u1, u2, wd);
                field_eval(&L, x, wd, Lw);
                const double V = output != 0 ? visibility(&L, x, wd) : 1.0;
                for (int c = 0; c < 3; ++c) acc[c] += wt * V * Lw[c];
            }
        for (int c = 0; c < 3; ++c) F[3 * p + c] = acc[c];
    }
    free(xs);
    free(ws);
}

/* ------------------------------------------------------------------------------------------ */
/* The paper's own cache input (Sec. "Neural Incident Radiance Cache": the list of encodings,
 * the amortised surface encoding, and the inference-pipeline figure, whose neural input vector
 * is 24 hash-grid + 25 spherical-harmonics + 3+8+4 surface values = 64):
 *   - x: multiresolution hash encoding (Mueller, Evans, Schied, Keller, "Instant neural graphics
 *     primitives with a multiresolution hash encoding", SIGGRAPH 2022), 12 levels of 2
 *     trainable features.  Level l has resolution N_l = floor(N_0 b^l); the position, clamped to
 *     the unit cube, is scaled by N_l; the 8 corners of its cell are looked up (a dense
 *     (N_l+1)^3 table when that fits in T entries, else the spatial hash
 *     (v0 * 1 xor v1 * 2654435761 xor v2 * 805459861) mod T) and blended trilinearly.
 *   - w: real spherical harmonics of degree <= 4 (25 values).
 *   - phi: shading normal (identity, 3), roughness as a one-blob encoding with 8 bins (Mueller,
 *     McWilliams, Rousselle, Gross, Novak, "Neural importance sampling", TOG 2019: a Gaussian of
 *     width 1/8 centred on the value, read at the bin centres), albedo (identity, 3; the white
 *     Lambertian surface has albedo 1) and one zero slot.
 * Canonical input order: hash (2 l + f), SH (l^2 + l + m), n, one-blob, albedo, zero.
 * Canonical parameter vector: W1 [W x 64], W2..W4 [W x W], W5 [3 x W] (row-major), then the
 * feature table, [entries][2], levels in order.                                               */
#define H_LEVELS 12
#define H_FEAT 2
#define H_IN 64
#define H_SH 25
#define H_MAX_LOG2T 24

typedef struct {
    int64_t T;
    int64_t res[H_LEVELS], size[H_LEVELS], off[H_LEVELS];
    int dense[H_LEVELS];
    int64_t entries;
} hgrid_t;

static void hgrid_setup(hgrid_t *g, int log2_table, int base_res, double growth)
{
    g->T = (int64_t)1 << log2_table;
    int64_t o = 0;
    for (int l = 0; l < H_LEVELS; ++l) {
        int64_t N = (int64_t)floor((double)base_res * pow(growth, (double)l));
        int64_t v = (N + 1) * (N + 1) * (N + 1);
        g->res[l] = N;
        g->dense[l] = v <= g->T;
        g->size[l] = g->dense[l] ? v : g->T;
        g->off[l] = o;
        o += g->size[l];
    }
    g->entries = o;
}

int64_t oracle_hash_entries(int log2_table, int base_res, double growth)
{
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
    return g.entries;
}

/* Resolution, first entry and dense flag of every level (for tests). */
void oracle_hash_levels(int log2_table, int base_res, double growth, int64_t *res, int64_t *off, int32_t *dense)
{
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
    for (int l = 0; l < H_LEVELS; ++l) {
        res[l] = g.res[l];
        off[l] = g.off[l];
        dense[l] = g.dense[l];
    }
}

/* Entry index (within the whole table) and trilinear weight of the 8 cell corners of x at level l. */
static void hash_corners(const hgrid_t *g, int l, const double x[3], int64_t idx[8], double wt[8])
{
    const int64_t N = g->res[l];
    int64_t c[3];
    double fr[3];
    for (int d = 0; d < 3; ++d) {
        double xc = x[d] < 0.0 ? 0.0 : (x[d] > 1.0 ? 1.0 : x[d]);
        double p = xc * (double)N;
        int64_t ci = (int64_t)floor(p);
        if (ci > N - 1) ci = N - 1;
        c[d] = ci;
        fr[d] = p - (double)ci;
    }
    for (int k = 0; k < 8; ++k) {
        int64_t v[3];
        double w = 1.0;
        for (int d = 0; d < 3; ++d) {
            int bit = (k >> d) & 1;
            v[d] = c[d] + bit;
            w *= bit ? fr[d] : 1.0 - fr[d];
        }
        int64_t i;
        if (g->dense[l]) {
            i = v[0] + (N + 1) * (v[1] + (N + 1) * v[2]);
        } else {
            uint32_t h = (uint32_t)v[0] * 1u ^ (uint32_t)v[1] * 2654435761u ^ (uint32_t)v[2] * 805459861u;
            i = (int64_t)(h % (uint32_t)g->T);
        }
        idx[k] = g->off[l] + i;
        wt[k] = w;
    }
}

static double factorial(int n)
{
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

/* Real spherical harmonics of degree <= 4 of the direction w (normalised here), without the
 * Condon-Shortley phase: index l^2 + l + m,
 *   m = 0: K_l^0 P_l(cos t);  m > 0: sqrt(2) K_l^m cos(m phi) P_l^m(cos t);
 *   m < 0: sqrt(2) K_l^|m| sin(|m| phi) P_l^|m|(cos t);  K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).
 * P_l^m from the standard recurrences: P_m^m = (2m-1)!! sin^m t, P_{m+1}^m = (2m+1) cos t P_m^m,
 * (l-m) P_l^m = (2l-1) cos t P_{l-1}^m - (l+m-1) P_{l-2}^m.                                     */
static void sh25(const double w_in[3], double Y[H_SH])
{
    double r = sqrt(w_in[0] * w_in[0] + w_in[1] * w_in[1] + w_in[2] * w_in[2]);
    double x = w_in[0] / r, y = w_in[1] / r, z = w_in[2] / r;
    double s = sqrt(x * x + y * y);
    double phi = atan2(y, x);
    double P[5][5];
    memset(P, 0, sizeof(P));
    for (int m = 0; m <= 4; ++m) {
        double pmm = 1.0;
        for (int k = 1; k <= m; ++k) pmm *= (2.0 * k - 1.0) * s;
        P[m][m] = pmm;
        if (m < 4) P[m + 1][m] = (2.0 * m + 1.0) * z * pmm;
        for (int l = m + 2; l <= 4; ++l)
            P[l][m] = ((2.0 * l - 1.0) * z * P[l - 1][m] - (double)(l + m - 1) * P[l - 2][m]) / (double)(l - m);
    }
    for (int l = 0; l <= 4; ++l)
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double v;
            if (m == 0) v = K * P[l][0];
            else if (m > 0) v = sqrt(2.0) * K * cos(m * phi) * P[l][m];
            else v = sqrt(2.0) * K * sin(am * phi) * P[l][am];
            Y[l * l + l + m] = v;
        }
}

void oracle_sh(int64_t Q, const double *dirs, double *Y)
{
    for (int64_t q = 0; q < Q; ++q) sh25(dirs + 3 * q, Y + H_SH * q);
}

/* One-blob encoding of v in [0,1] with 8 bins: exp(-((v - (i + 1/2)/8) / (1/8))^2 / 2). */
static void oneblob8(double v, double out[8])
{
    for (int i = 0; i < 8; ++i) {
        double d = (v - (i + 0.5) / 8.0) * 8.0;
        out[i] = exp(-0.5 * d * d);
    }
}

/* The 64 inputs of point p and direction w; the table holds [entries][2] features. */
static void hash_inputs(const hgrid_t *g, const double *table, const float *const pts[7], int64_t p,
                        const double w[3], double e[H_IN])
{
    double x[3] = {pts[0][p], pts[1][p], pts[2][p]};
    for (int l = 0; l < H_LEVELS; ++l) {
        int64_t idx[8];
        double wt[8];
        hash_corners(g, l, x, idx, wt);
        for (int f = 0; f < H_FEAT; ++f) {
            double s = 0.0;
            for (int k = 0; k < 8; ++k) s += wt[k] * table[2 * idx[k] + f];
            e[2 * l + f] = s;
        }
    }
    sh25(w, e + 24);
    e[49] = pts[3][p];
    e[50] = pts[4][p];
    e[51] = pts[5][p];
    oneblob8(pts[6][p], e + 52);
    e[60] = e[61] = e[62] = 1.0;
    e[63] = 0.0;
}

static int64_t hash_mlp_params(int width) { return (int64_t)width * H_IN + 3LL * width * width + 3LL * width; }

int64_t oracle_hash_n_params(int width, int log2_table, int base_res, double growth)
{
    return hash_mlp_params(width) + 2 * oracle_hash_entries(log2_table, base_res, growth);
}

static void hash_net_setup(net_t *net, const double *w, int width)
{
    net->width = width;
    net->vis = 0;
    int rows[5] = {width, width, width, width, 3};
    int cols[5] = {H_IN, width, width, width, width};
    size_t off = 0;
    for (int l = 0; l < 5; ++l) {
        net->W[l] = w + off;
        net->rows[l] = rows[l];
        net->cols[l] = cols[l];
        off += (size_t)rows[l] * cols[l];
    }
}

void oracle_hash_encode(int64_t Q, const float *px, const float *py, const float *pz, const float *nx,
                        const float *ny, const float *nz, const float *rough, const int32_t *point,
                        const double *dirs, const double *table, int log2_table, int base_res, double growth,
                        double *e /* [Q][64] */)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) hash_inputs(&g, table, pts, point ? point[q] : q, dirs + 3 * q, e + H_IN * q);
}

void oracle_hash_infer(int64_t Q, const float *px, const float *py, const float *pz, const float *nx,
                       const float *ny, const float *nz, const float *rough, const int32_t *point,
                       const double *dirs, const double *w, int width, int log2_table, int base_res,
                       double growth, double *rgb)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
    net_t net;
    hash_net_setup(&net, w, width);
    const double *table = w + hash_mlp_params(width);
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < Q; ++q) {
        double e[H_IN];
        acts_t a;
        hash_inputs(&g, table, pts, point ? point[q] : q, dirs + 3 * q, e);
        net_forward(&net, e, &a);
        for (int c = 0; c < 3; ++c) rgb[3 * q + c] = a.y[c];
    }
}

/* The two-level estimator of the radiance cache on this input (the same three sums as for the
 * frequency input; directions sampled here, or given as [P][N+1][3]). */
void oracle_hash_estimate(int64_t P, const float *px, const float *py, const float *pz, const float *nx,
                          const float *ny, const float *nz, const float *rough, const float *lobes,
                          const double *w, int width, int log2_table, int base_res, double growth, int n_cache,
                          uint64_t seed, uint64_t frame, const double *dirs, const double *residual_radiance,
                          double *out_tl, double *out_c, double *out_r)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    lobes_t L;
    lobes_unpack(lobes, &L);
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
    net_t net;
    hash_net_setup(&net, w, width);
    const double *table = w + hash_mlp_params(width);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t p = 0; p < P; ++p) {
        double x[3] = {px[p], py[p], pz[p]};
        double n[3] = {nx[p], ny[p], nz[p]};
        double fc[3] = {0, 0, 0}, fr[3];
        for (int k = 0; k <= n_cache; ++k) {
            double wdir[3];
            if (dirs) {
                const double *d = dirs + ((size_t)p * (n_cache + 1) + k) * 3;
                wdir[0] = d[0]; wdir[1] = d[1]; wdir[2] = d[2];
            } else {
                double u1, u2;
                direction_uniforms(seed, (uint32_t)p, k, k == n_cache, (uint32_t)frame, &u1, &u2);
                cosine_direction(n, u1, u2, wdir);
            }
            double e[H_IN];
            acts_t a;
            hash_inputs(&g, table, pts, p, wdir, e);
            net_forward(&net, e, &a);
            if (k < n_cache) {
                for (int c = 0; c < 3; ++c) fc[c] += a.y[c];
            } else {
                double Lw[3];
                if (residual_radiance) {
                    for (int c = 0; c < 3; ++c) Lw[c] = residual_radiance[3 * p + c];
                } else {
                    field_eval(&L, x, wdir, Lw);
                }
                for (int c = 0; c < 3; ++c) fr[c] = Lw[c] - a.y[c];
            }
        }
        for (int c = 0; c < 3; ++c) {
            double Fc = fc[c] / n_cache;
            if (out_c) out_c[3 * p + c] = Fc;
            if (out_r) out_r[3 * p + c] = fr[c];
            if (out_tl) out_tl[3 * p + c] = Fc + fr[c];
        }
    }
}

/* Loss and gradient of the hash-input cache (kind 0 relative L2 with the denominator held
 * constant unless frozen == 0, kind 1 plain L2), as for the frequency input; in addition the
 * gradient reaches the inputs of the hash features, dloss/de_k = sum_r W1[r][k] delta1[r], and
 * each table entry receives the trilinear weight of its corner times that (the scatter of the
 * interpolation's transpose).  grad: [n_params] in canonical order (MLP, then table).
 * ReLU'(0) = 0: a unit whose pre-activation is exactly zero passes no gradient.          */
double oracle_hash_loss_grad(int64_t B, const float *px, const float *py, const float *pz, const float *nx,
                             const float *ny, const float *nz, const float *rough, const int32_t *point,
                             const double *dirs, const double *target, const double *w, int width,
                             int log2_table, int base_res, double growth, double eps, int frozen, int kind,
                             double *grad)
{
    const float *pts[7] = {px, py, pz, nx, ny, nz, rough};
    hgrid_t g;
    hgrid_setup(&g, log2_table, base_res, growth);
    net_t net;
    hash_net_setup(&net, w, width);
    const int W = width;
    const int64_t nm = hash_mlp_params(W), nt = 2 * g.entries;
    const double *table = w + nm;
    if (grad) memset(grad, 0, sizeof(double) * (size_t)(nm + nt));
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *tg = grad ? (double *)calloc((size_t)nthreads * nm, sizeof(double)) : NULL;
    double *tl = (double *)calloc((size_t)nthreads, sizeof(double));
    double *de = grad ? (double *)calloc((size_t)B * 24, sizeof(double)) : NULL;   /* dloss/d(hash inputs) */
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gm = tg ? tg + (size_t)tid * nm : NULL;
#pragma omp for schedule(static)
        for (int64_t b = 0; b < B; ++b) {
            double e[H_IN];
            acts_t a;
            hash_inputs(&g, table, pts, point ? point[b] : b, dirs + 3 * b, e);
            net_forward(&net, e, &a);
            double dz[3];
            for (int c = 0; c < 3; ++c) {
                double y = a.y[c], t = target[3 * b + c];
                double d = y - t;
                double den = (kind == 0) ? y * y + eps : 1.0;
                tl[tid] += d * d / den;
                double dy = 2.0 * d / den;
                if (!frozen && kind == 0) dy -= d * d * 2.0 * y / (den * den);
                dz[c] = dy * y / (3.0 * (double)B);
            }
            if (!gm) continue;
            double *gW5 = gm + (size_t)W * H_IN + 3LL * W * W;
            for (int c = 0; c < 3; ++c)
                for (int j = 0; j < W; ++j) gW5[(size_t)c * W + j] += dz[c] * a.h[3][j];
            double delta[256], prev[256];
            for (int j = 0; j < W; ++j) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c) s += net.W[4][(size_t)c * W + j] * dz[c];
                delta[j] = a.z[3][j] > 0.0 ? s : 0.0;
            }
            for (int l = 3; l >= 1; --l) {
                double *gW = gm + (size_t)W * H_IN + (size_t)(l - 1) * W * W;
                for (int r = 0; r < W; ++r)
                    for (int c = 0; c < W; ++c) gW[(size_t)r * W + c] += delta[r] * a.h[l - 1][c];
                for (int c = 0; c < W; ++c) {
                    double s = 0.0;
                    for (int r = 0; r < W; ++r) s += net.W[l][(size_t)r * W + c] * delta[r];
                    prev[c] = a.z[l - 1][c] > 0.0 ? s : 0.0;
                }
                memcpy(delta, prev, sizeof(double) * W);
            }
            for (int r = 0; r < W; ++r)
                for (int c = 0; c < H_IN; ++c) gm[(size_t)r * H_IN + c] += delta[r] * e[c];
            for (int k = 0; k < 24; ++k) {
                double s = 0.0;
                for (int r = 0; r < W; ++r) s += net.W[0][(size_t)r * H_IN + k] * delta[r];
                de[24 * b + k] = s;
            }
        }
    }
    double loss = 0.0;
    for (int t = 0; t < nthreads; ++t) loss += tl[t];
    if (grad) {
        for (int t = 0; t < nthreads; ++t)
            for (int64_t i = 0; i < nm; ++i) grad[i] += tg[(size_t)t * nm + i];
        double *gt = grad + nm;
        for (int64_t b = 0; b < B; ++b) {
            int64_t p = point ? point[b] : b;
            double x[3] = {px[p], py[p], pz[p]};
            for (int l = 0; l < H_LEVELS; ++l) {
                int64_t idx[8];
                double wt[8];
                hash_corners(&g, l, x, idx, wt);
                for (int k = 0; k < 8; ++k)
                    for (int f = 0; f < H_FEAT; ++f) gt[2 * idx[k] + f] += wt[k] * de[24 * b + 2 * l + f];
            }
        }
    }
    free(tg);
    free(tl);
    free(de);
    return loss / (3.0 * (double)B);
}
