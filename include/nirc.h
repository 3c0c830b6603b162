/*
 * nirc.h - C ABI of the MI355X (gfx950) library for the neural incident radiance cache (NIRC)
 * and the two-level Monte Carlo estimator built on it.
 *
 * The method (Sec. "Neural Incident Radiance Cache"):
 *   - the cache n(x, w, phi; W) is a small MLP that predicts incident radiance at a shading point
 *     x with features phi (normal, roughness) for an incident direction w (eq. 11);
 *   - the two-level estimator of the reflected radiance is
 *       L_o = L_c + L_r  (eq. L_mlmc, emission omitted),
 *       L_c = (1/N) sum_k n(x, w_k) f_r cos / p       over N cache directions   (eq. L_c),
 *       L_r = (L_i(x, w_r) - n(x, w_r)) f_r cos / p   over one independent direction (eq. L_r),
 *     which is unbiased whatever the cache weights are (eq. Fc, Fr, Fml);
 *   - the cache is trained online, several Adam steps per frame, with a relative L2 loss whose
 *     denominator is excluded from differentiation (eq. 12).
 * The library uses a white Lambertian BRDF (f_r = 1/pi) with cosine-weighted directions, so
 * f_r cos / p = 1: L_c is the mean of the N cache predictions and L_r is target minus cache.
 *
 * Network: 10 inputs (x[3], w[3], n[3], roughness) -> sin/cos(2^k pi v), k = 0..7 -> 160
 * features -> 4 hidden ReLU layers of `width` -> 3 outputs -> exp.  No biases.  Canonical
 * parameter vector (FP32, row-major per layer, layers concatenated): W1 [width x 160],
 * W2, W3, W4 [width x width], W5 [3 x width]; feature 16*i + 2*k + (0 sin | 1 cos) of input i
 * in the order (x0, x1, x2, w0, w1, w2, n0, n1, n2, roughness).
 *
 * Conventions for every entry point:
 *   - pointers are DEVICE pointers unless the comment says host; the caller owns all memory
 *     (model state and workspace included) and the library never allocates device memory;
 *   - every call only enqueues work on `stream` (a hipStream_t; NULL = the null stream) and
 *     returns without synchronising;
 *   - argument and shape errors are reported synchronously, before anything is enqueued, as a
 *     negative nirc_status; a failed kernel launch returns NIRC_ERR_HIP;
 *   - numeric faults in training (a non-finite loss or gradient) never trap: the Adam update is
 *     skipped on the device and a flag is raised (nirc_read_flags);
 *   - one model must not be used on two streams at once; distinct models may run concurrently.
 */
#ifndef NIRC_H
#define NIRC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nirc_status;
#define NIRC_OK 0
#define NIRC_ERR_INVALID_ARG (-1)
#define NIRC_ERR_UNSUPPORTED (-2)
#define NIRC_ERR_WORKSPACE (-3)   /* state or workspace buffer too small */
#define NIRC_ERR_HIP (-5)

/* Arithmetic of the MLP layer products (FP32 accumulation in every case). */
#define NIRC_FP32 0
#define NIRC_BF16 1
#define NIRC_FP16 2

/* Training loss (Sec. "Radiance Cache Optimization"), per sample and channel with d = y - t:
 *   NIRC_LOSS_REL_L2  d^2 / (sg(y)^2 + loss_eps)         eq. 12, the method's loss (default);
 *   NIRC_LOSS_L2      d^2                                 the plain squared difference;
 *   NIRC_LOSS_VAR     (t - y - F_r)^2                     the residual-variance loss, with F_r the
 *                     batch mean of t - y per channel (computed by a forward pass first).
 * The loss is the mean over samples and channels; the training direction pdf is taken as 1. */
#define NIRC_LOSS_REL_L2 0
#define NIRC_LOSS_L2 1
#define NIRC_LOSS_VAR 2

/* What the cache learns and which scene it sees (Sec. "Neural Visibility Cache").
 *   NIRC_OUTPUT_RADIANCE           exp outputs predict incident radiance; the scene is the
 *                                  field alone (the default).
 *   NIRC_OUTPUT_VISIBILITY         the visibility cache: sigmoid outputs predict the visibility V
 *                                  in [0, 1]; incident radiance is V times the known radiance
 *                                  L (the field, standing in for an environment map), so the
 *                                  estimator's cache level uses n_V(x, w) L(x, w), training
 *                                  targets are V, and the residual sample is V L.
 *   NIRC_OUTPUT_RADIANCE_OCCLUDED  a radiance cache (exp outputs) on the same occluded scene:
 *                                  targets and residual samples are V L (the comparison case).
 * The synthetic occluder: V(x, w) = 1 - 0.9 / (1 + exp(-16 (mu_0 . w - c(x)))), c(x) = 0.6 +
 * 0.3 (x_0 - 0.5), with mu_0 the field's first lobe axis (a soft cap blocking 90 % of it). */
#define NIRC_OUTPUT_RADIANCE 0
#define NIRC_OUTPUT_VISIBILITY 1
#define NIRC_OUTPUT_RADIANCE_OCCLUDED 2

/* Device flags of a model (sticky until nirc_clear_flags). */
#define NIRC_FLAG_NONFINITE_GRAD 1u   /* a step saw a non-finite loss/gradient and was skipped */
#define NIRC_FLAG_BAD_POINT_INDEX 2u  /* a query named a point index outside [0, points.count):
                                         in training the step was skipped; in inference that
                                         query's outputs are not defined */

typedef struct nirc_model nirc_model;   /* opaque host handle */

/* Host struct.  Adam hyper-parameters follow Kingma & Ba; the paper trains with Adam, several
 * steps per frame (Sec. "Results").  loss_eps is the epsilon of the relative L2 loss (eq. 12).
 * loss_scale multiplies the loss before the backward pass and divides the gradient after it; for
 * BF16 and FP16 models it is taken per sample (times the batch size, so that 16-bit deltas stay
 * near unit size).  FP16 models scale dynamically: loss_scale is the starting value, a training
 * step skipped for a non-finite gradient halves the scale, 1000 finite steps in a row double it
 * (within [2^-14, 2^24]); nirc_read_loss_scale returns the current value, and the training state
 * (nirc_get_state) carries it. */
typedef struct {
    int32_t width;       /* hidden width: 64 or 128 (the batched estimator: 64 only) */
    int32_t precision;   /* NIRC_FP32 | NIRC_BF16 | NIRC_FP16 */
    float lr;            /* e.g. 1e-3 */
    float beta1;         /* e.g. 0.9 */
    float beta2;         /* e.g. 0.999 */
    float adam_eps;      /* e.g. 1e-8 */
    float loss_eps;      /* e.g. 1e-2 */
    float loss_scale;    /* e.g. 1 (FP32/BF16); > 1 for FP16 */
    int32_t loss;        /* NIRC_LOSS_REL_L2 | NIRC_LOSS_L2 | NIRC_LOSS_VAR */
    int32_t output;      /* NIRC_OUTPUT_RADIANCE | NIRC_OUTPUT_VISIBILITY | NIRC_OUTPUT_RADIANCE_OCCLUDED */
} nirc_config;

/* Shading points, structure of arrays, FP32 device arrays of `count` entries each. */
typedef struct {
    const float *px, *py, *pz;   /* position */
    const float *nx, *ny, *nz;   /* unit normal */
    const float *rough;          /* roughness */
    int64_t count;
} nirc_points;

/* Cache queries: a direction per query and the index of its shading point (point == NULL
 * means query i uses point i).  FP32 / int32 device arrays of `count` entries.  A point index
 * outside [0, points.count) is an error found on the device: the kernels never read out of
 * bounds for it, raise NIRC_FLAG_BAD_POINT_INDEX in the model's flags (training skips the step,
 * inference leaves that query's outputs undefined) and nirc_encode writes NaN features for it. */
typedef struct {
    const float *wx, *wy, *wz;
    const int32_t *point;
    int64_t count;
} nirc_queries;

/* Synthetic incident radiance field standing in for path-traced radiance (host struct, passed
 * by pointer and copied at the call): L_c(x, w) = sum_j a_jc(x) exp(kappa_j (mu_j . w - 1)),
 * a_jc(x) = alpha_jc + sum_d beta_jcd x_d.  The record is 64 floats in this order. */
typedef struct {
    float axis[4][3];
    float kappa[4];
    float alpha[4][3];
    float beta[4][3][3];
} nirc_lobes;

/* ------------------------------------------------------------------------------------------ */
/* Sizes and model lifetime                                                                   */

/* Number of parameters of the canonical vector: width*160 + 3*width^2 + 3*width; 0 if the
 * width is unsupported. */
int64_t nirc_n_params(int32_t width);

/* Bytes of model state (FP32 master weights, Adam moments, step counter, flags and the packed
 * copy the kernels read).  0 if the configuration is invalid. */
size_t nirc_state_bytes(const nirc_config *cfg /* host */);

/* Bytes of workspace needed by training calls on batches of up to max_batch queries
 * (per-workgroup gradient partials, reduced gradient, loss, and the sample buffers of
 * nirc_train_frame, which makes the samples of up to 4 steps in one launch).  Inference needs
 * none. */
size_t nirc_workspace_bytes(const nirc_config *cfg /* host */, int64_t max_batch);

/* Create a model over caller-owned device buffers.  `state` must hold nirc_state_bytes and be
 * 256-byte aligned; `workspace` may be NULL (no training) or hold nirc_workspace_bytes(cfg, B).
 * `init_w` is the canonical FP32 parameter vector (device).  Adam moments and the step counter
 * start at zero.  *out receives a host handle, freed by nirc_destroy (which frees no device
 * memory). */
nirc_status nirc_create(const nirc_config *cfg /* host */, void *state, size_t state_bytes,
                        void *workspace, size_t workspace_bytes, const float *init_w,
                        void *stream, nirc_model **out /* host */);
nirc_status nirc_destroy(nirc_model *model);

/* Replace the weights (canonical FP32, device) and reset Adam (moments and step). */
nirc_status nirc_set_weights(nirc_model *model, const float *w, void *stream);
/* Copy the FP32 master weights to `w` (canonical, device). */
nirc_status nirc_get_weights(const nirc_model *model, float *w, void *stream);
/* Copy the Adam state: m and v (canonical FP32, device, may be NULL) and the step counter
 * (device int64, may be NULL). */
nirc_status nirc_get_adam(const nirc_model *model, float *m, float *v, int64_t *step, void *stream);

/* The whole training state (FP32 weights, Adam moments and step, packed copies, flags) as one
 * device blob of nirc_state_bytes(cfg) bytes, for checkpoint and resume.  nirc_set_state takes
 * a blob written by nirc_get_state of a model of the same width (blob_bytes must equal this
 * model's state size) and re-derives the packed copies from its FP32 weights, so a resumed
 * model continues exactly as the saved one would have.  Both only enqueue device copies on
 * `stream`; the blob belongs to the caller. */
nirc_status nirc_get_state(const nirc_model *model, void *blob, size_t blob_bytes, void *stream);
nirc_status nirc_set_state(nirc_model *model, const void *blob, size_t blob_bytes, void *stream);

/* Sticky device flags (NIRC_FLAG_*).  Reads them synchronously on `stream` (host call that
 * waits for the stream); returns 0xFFFFFFFF on error. */
uint32_t nirc_read_flags(const nirc_model *model, void *stream);
nirc_status nirc_clear_flags(nirc_model *model, void *stream);

/* The model's current loss scale (the dynamic one of FP16 models, else loss_scale); reads it
 * synchronously on `stream`; -1 on error. */
float nirc_read_loss_scale(const nirc_model *model, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Inference                                                                                   */

/* The 160 input features of each query (Sec. "Neural Network Architecture": the network sees
 * an encoding of the position, the direction and the surface features).  features is
 * [queries.count][160] FP32 in canonical feature order. */
nirc_status nirc_encode(nirc_points points, nirc_queries queries, float *features, void *stream);

/* Cache predictions n(x, w) for explicit queries (eq. 11's network term): rgb is
 * [queries.count][3] FP32.  Every query is evaluated independently (no sharing of the surface
 * encoding between queries of one point). */
nirc_status nirc_infer(const nirc_model *model, nirc_points points, nirc_queries queries,
                       float *rgb, void *stream);

/* The sampled directions the estimator uses (Sec. "Cache application": independent BSDF
 * sampling for the cache and the residual).  dirs is [points.count][n_cache + 1][3] FP32; entry
 * n_cache of each point is the residual direction.  Cosine-weighted about the normal, from
 * Philox4x32-10 with key (seed lo, seed hi): cache direction k of point p uses counter
 * (p, k >> 1, frame, 3), words (0,1) for even k and (2,3) for odd k; the residual direction of
 * p uses counter (p >> 1, 0, frame, 4), words (0,1) for even p and (2,3) for odd p.  A word r
 * gives u = (r >> 8) 2^-24. */
nirc_status tlmc_sample_dirs(nirc_points points, int32_t n_cache, uint64_t seed, uint64_t frame,
                             float *dirs, void *stream);

/* The two-level estimator per shading point and channel (eq. L_mlmc, L_c, L_r):
 *   out_c  = (1/N) sum_k n(x, w_k)         (cache level, N = n_cache >= 1)
 *   out_r  = L(x, w_r) - n(x, w_r)          (residual)
 *   out_tl = out_c + out_r
 * Directions are generated in the kernel as tlmc_sample_dirs returns them: exactly for the FP32
 * model and for every residual direction; the 16-bit models' cache directions take the
 * hardware sine of the same uniforms (within ~1e-6 of the sampler's, far below their 16-bit
 * operands; they never leave the kernel).  The
 * surface part of the first layer is computed once per point and shared by its N + 1 queries
 * (Sec. "Neural Network Architecture": amortised surface encoding).
 * L(x, w_r) is the residual sample's radiance (Sec. "Cache application": one path-traced
 * sample per shading point): residual_radiance ([points.count][3] FP32) when given — a
 * renderer traces the residual directions tlmc_sample_dirs returns (entry n_cache of each
 * point) and passes what it found — otherwise the synthetic lobe field `field` evaluated in the
 * kernel (then `field` may be NULL).  out_c and out_r may be NULL.  All outputs are [points.count][3] FP32. */
nirc_status tlmc_estimate(const nirc_model *model, nirc_points points,
                          const nirc_lobes *field /* host */, int32_t n_cache, uint64_t seed,
                          uint64_t frame, const float *residual_radiance /* nullable */,
                          float *out_tl, float *out_c, float *out_r, void *stream);

/* The biased estimator with the Balanced Termination Heuristic at the shading point (Sec. "Path
 * Termination Heuristics", first path vertex).  The path's scattering direction w_s is drawn from
 * the BRDF (cosine-weighted, pdf p = cos/pi) — it is the residual direction of tlmc_estimate,
 * entry n_cache of tlmc_sample_dirs — and continues with probability
 *   P_s = p / (p + N/pi) = cos / (cos + N):
 * a uniform xi (Philox counter (p >> 2, 0, frame, 6), word p & 3) stops the path if xi > P_s,
 * and the point is then shaded by the N cache samples alone, out = F_c; otherwise the path goes
 * on and its radiance L(x, w_s) is the estimate (residual_radiance when given — the renderer
 * traces the continued paths — else the field).  The decision is exact: with cos = sqrt(1 - u1)
 * and the 24-bit uniforms xi = X 2^-24, u1 = U 2^-24 it is (X N)^2 2^24 > (2^24 - U)(2^24 - X)^2
 * in 128-bit integers.
 * out_b [points.count][3]; out_c [points.count][3] (required: F_c); out_continue
 * [points.count] int32, 1 where the path continues (nullable). */
nirc_status tlmc_estimate_biased(const nirc_model *model, nirc_points points,
                                 const nirc_lobes *field /* host */, int32_t n_cache, uint64_t seed,
                                 uint64_t frame, const float *residual_radiance /* nullable */,
                                 float *out_b, float *out_c, int32_t *out_continue, void *stream);

/* The estimator with the fusions of the paper's inference pipeline undone, for measuring what
 * each buys (Sec. "Neural Network Architecture": the pipeline comparison of shared surface
 * encodings, the direction encoding fused into the network, and direct output from on-chip
 * memory).  Every stage computes the estimate of tlmc_estimate (same directions and features;
 * sums in another order):
 *   stage 0: one kernel writes every query's 160 encoded inputs (16-bit MFMA operands) to the
 *            workspace, the network kernel reads them and writes one prediction per query, a
 *            third kernel forms F_c, F_r and F_tl per point;
 *   stage 1: as 0, the surface inputs encoded once per point and shared by its N + 1 queries;
 *   stage 2: as 1, the directions drawn and encoded inside the network kernel;
 *   stage 3: tlmc_estimate itself.
 * BF16 / FP16 models of width 64 with NIRC_OUTPUT_RADIANCE; the field is required.  workspace:
 * 256-byte aligned, tlmc_unfused_workspace_bytes (0 for stage 3, and for invalid arguments or
 * more than 2^32 queries). */
size_t tlmc_unfused_workspace_bytes(int64_t points, int32_t n_cache, int32_t stage);
nirc_status tlmc_estimate_unfused(const nirc_model *model, nirc_points points, const nirc_lobes *field /* host */,
                                  int32_t n_cache, uint64_t seed, uint64_t frame, int32_t stage, void *workspace,
                                  size_t workspace_bytes, float *out_tl, float *out_c, float *out_r, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Continuous batching of estimates (several render streams, each with its own cache)         */

#define TLMC_BATCH_MAX_REQUESTS 64

/* One frame of one render stream: its model, points, field or residual radiance, sample count,
 * seed and frame, and where the results go (as for tlmc_estimate).  Host struct. */
typedef struct {
    const nirc_model *model;
    nirc_points points;
    nirc_lobes field;
    int32_t n_cache;
    uint64_t seed;
    uint64_t frame;
    const float *residual_radiance;   /* NULL: the field */
    float *out_tl, *out_c, *out_r;
} tlmc_request;

/* Bytes of a work list. */
size_t tlmc_batch_bytes(void);

/* Fill a work list (host memory of tlmc_batch_bytes) for n requests (1..TLMC_BATCH_MAX_REQUESTS)
 * whose models share width, precision and output mode.  The caller copies it to device memory and launches
 * tlmc_estimate_batch on it; the list only holds device pointers, so it stays valid as long as
 * the models and buffers it names do. */
nirc_status tlmc_batch_build(const tlmc_request *requests /* host */, int32_t n, void *list /* host */);

/* Every request of a device work list in one persistent launch: a fixed grid walks the list in
 * chunks of 128 points, re-staging weights only when the request changes.  Results are identical
 * to tlmc_estimate of each request alone.  The launch shape does not depend on the list, so a
 * captured launch (hipGraph) can be replayed after writing a different list to the same buffer.
 * width, precision and output (NIRC_OUTPUT_*) must match the list's models. */
nirc_status tlmc_estimate_batch(const void *list /* device */, int32_t width, int32_t precision, int32_t output,
                                void *stream);

/* Continuous batching of online training (several render streams, each with its own cache): one
 * frame's training of each request of a work list, every step of all requests in one set of
 * launches (samples, gradient, reduction, Adam with the 16-bit refresh), so that a frame loop
 * over many streams can replay one captured graph for the whole mix.  Host struct. */
#define NIRC_TRAIN_BATCH_MAX_REQUESTS 64
typedef struct {
    nirc_model *model;     /* width 64, NIRC_BF16 or NIRC_FP16, loss other than NIRC_LOSS_VAR, created
                              with a workspace of nirc_workspace_bytes(cfg, >= batch); at most once per list */
    nirc_points points;
    nirc_lobes field;      /* the frame's field (the training targets) */
    int64_t batch;         /* samples per step, 1..max_batch */
    uint64_t seed;
    uint64_t frame;
} nirc_train_request;

/* Bytes of a training work list. */
size_t nirc_train_list_bytes(void);

/* Fill a training work list (host memory of nirc_train_list_bytes) for n requests
 * (1..NIRC_TRAIN_BATCH_MAX_REQUESTS) whose models share width and precision; the caller copies it
 * to device memory.  The list holds device pointers only (models, their workspaces, points). */
nirc_status nirc_train_list_build(const nirc_train_request *requests, int32_t n, int64_t max_batch,
                                  void *list /* host */);

/* `steps` training steps of every request of a device work list: step s of request r is
 * nirc_train_frame(model, points, field, batch, steps, seed, frame)'s step s, with bit-identical
 * results (same samples, same gradient blocks, same reduction order; each model's own workspace),
 * and the steps of all requests run together.  Losses are not returned.  precision must be the
 * list's; max_batch bounds the list's batches and fixes the launch shapes, which do not depend on
 * the list: a captured sequence can be replayed after writing another list to the same buffer. */
nirc_status nirc_train_frame_batch(const void *list /* device */, int32_t steps, int32_t precision,
                                   int64_t max_batch, void *stream);

/* Reference integral of the occluded scene, F(x) = (1/pi) int V(x, w) L(x, w) (n . w) dw, by
 * tensor Gauss-Legendre quadrature with n_nodes (8..128) nodes per axis over the two uniforms of
 * the cosine-weighted map (whose pdf cancels the cosine); FP32 integrand, FP64 sums.  F is
 * [points.count][3] FP64.  A measurement reference (the occluded integral has no closed form). */
nirc_status tlmc_reference_occluded(nirc_points points, const nirc_lobes *field /* host */, int32_t n_nodes,
                                    double *F, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Training                                                                                    */

/* Training samples (stand-in for the paper's separate training pass, Sec. "Cache
 * application"): sample b of step `step` in `frame` draws Philox counter (b, step, frame, 5):
 * word 0 picks the point floor(r0 * count / 2^32), words 1 and 2 a cosine-weighted direction
 * about its normal; the target is what a cache of kind `output` learns there (NIRC_OUTPUT_*):
 * the field's radiance L, the visibility V (in every channel) or V L.  Outputs: point [batch]
 * int32, wx, wy, wz [batch] FP32 and target [batch][3] FP32. */
nirc_status tlmc_train_batch(nirc_points points, const nirc_lobes *field /* host */, int64_t batch,
                             uint64_t seed, uint64_t frame, uint32_t step, int32_t output, int32_t *point,
                             float *wx, float *wy, float *wz, float *target, void *stream);

/* Gradient of the relative L2 loss (eq. 12, on radiance, stop-gradient denominator):
 *   loss = (1/(3B)) sum_{b,c} (y - t)^2 / (sg(y)^2 + loss_eps)
 * w.r.t. the weights, written to grad [n_params] (canonical FP32); loss (device float, may be
 * NULL) receives the loss.  Needs the workspace.  Deterministic (fixed reduction order).
 * FP32 models run FP32 MFMA; BF16 / FP16 models run the forward and backward with 16-bit
 * operands and FP32 accumulation, with the output gradient scaled by loss_scale * B before the
 * backward and the gradient unscaled after the reduction.  Width 128 sweeps the batch several
 * times (each sweep owns a disjoint part of the gradient). */
nirc_status nirc_loss_grad(nirc_model *model, nirc_points points, nirc_queries queries,
                           const float *target, float *grad, float *loss, void *stream);

/* Vector-Jacobian product for automatic differentiation: grad = d(sum_q,c d_rgb[q][c] *
 * y[q][c]) / dW for the predictions y of nirc_infer.  Needs the workspace. */
nirc_status nirc_backward(nirc_model *model, nirc_points points, nirc_queries queries,
                          const float *d_rgb, float *grad, void *stream);

/* One Adam step with the given gradient (canonical FP32); skipped, with
 * NIRC_FLAG_NONFINITE_GRAD raised, if any gradient entry is not finite. */
nirc_status nirc_adam_step(nirc_model *model, const float *grad, void *stream);

/* nirc_loss_grad followed by nirc_adam_step on the workspace gradient. */
nirc_status nirc_train_step(nirc_model *model, nirc_points points, nirc_queries queries,
                            const float *target, float *loss, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): nirc_train_step with its scratch (gradient partials,
 * the reduced gradient, the loss, the residual-variance pre-pass) in a static device buffer of
 * the library (9.3 MB per GPU, held until the process ends) instead of the model's workspace, so
 * a model created without workspace can train.  Allocates nothing: no hipMalloc, no library
 * allocation.  queries.count must be 1..NIRC_STATIC_MAX_BATCH (else NIRC_ERR_INVALID_ARG,
 * before anything is enqueued).  Every call on one GPU shares that GPU's buffer: calls that
 * overlap on one GPU (two streams, or two host threads) race and must be serialised by the
 * caller.  Results are identical to nirc_train_step's on the same inputs. */
#define NIRC_STATIC_MAX_BATCH 2048
nirc_status nirc_train_step_static(nirc_model *model, nirc_points points, nirc_queries queries,
                                   const float *target, float *loss, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Frame statistics (FP64 on the device)                                                       */

/* Coefficients per lobe of the Chebyshev expansion used for the ground truth. */
#define TLMC_CHEB_COEFFS 128
/* Doubles written by tlmc_frame_stats. */
#define TLMC_STATS 8

/* Ground truth of the estimator for the lobe field with f_r = 1/pi (the quantity eq. L_mlmc
 * estimates, emission omitted): F(x, n) = sum_j a_j(x) J(kappa_j, mu_j . n), where
 * J(kappa, t) = (1/pi) int_{H+} exp(kappa (mu . w - 1)) cos(theta) dw reduces to a 1D integral
 * with a modified Bessel function.  tlmc_reference_table builds, for each lobe, a Chebyshev
 * expansion of J(kappa_j, .) on [-1, 1] by Gauss-Legendre quadrature: table is
 * [4][TLMC_CHEB_COEFFS] FP64 (device) and depends only on the kappas, so a scene whose lobes
 * rotate keeps its table. */
nirc_status tlmc_reference_table(const nirc_lobes *field /* host */, double *table, void *stream);

/* F per point: [points.count][3] FP64. */
nirc_status tlmc_reference(nirc_points points, const nirc_lobes *field /* host */, const double *table,
                           double *F, void *stream);

/* Bytes of scratch tlmc_frame_stats needs. */
size_t tlmc_frame_stats_scratch_bytes(void);

/* Per-frame error statistics of an estimate against F, summed in FP64 in a fixed order:
 *   stats[0] = sum (F_tl - F)^2 / (F^2 + eps)    stats[4] = stats[0] / stats[3]  (MRSE)
 *   stats[1] = sum (F_c  - F)^2 / (F^2 + eps)    stats[5] = stats[1] / stats[3]
 *   stats[2] = sum  F_r^2       / (F^2 + eps)    stats[6] = stats[2] / stats[3]
 *   stats[3] = number of terms (3 * points.count)
 * over points and channels (est_c / est_r may be NULL: their sums are 0).  The paper reports
 * the mean relative squared error (MRSE) without defining it; this is the usual form with
 * eps guarding dark pixels. */
nirc_status tlmc_frame_stats(nirc_points points, const nirc_lobes *field /* host */, const double *table,
                             const float *est_tl, const float *est_c, const float *est_r, double eps,
                             void *scratch, double *stats /* [TLMC_STATS] */, void *stream);

/* sum[i] += v[i], sumsq[i] += v[i]^2 in FP64 (per-point accumulation over seeds). */
nirc_status tlmc_accumulate(const float *values, int64_t count, double *sum, double *sumsq, void *stream);

/* One frame's online training (Sec. "Results": several Adam steps per frame on samples of a
 * separate training pass): for step s = 0..steps-1, tlmc_train_batch(points, field, batch, seed,
 * frame, s) into the workspace, then nirc_train_step on it.  The workspace must hold
 * nirc_workspace_bytes(cfg, batch).  loss (device float, may be NULL) receives the last step's
 * loss. */
nirc_status nirc_train_frame(nirc_model *model, nirc_points points, const nirc_lobes *field /* host */,
                             int64_t batch, int32_t steps, uint64_t seed, uint64_t frame, float *loss,
                             void *stream);

/* ==========================================================================================
 * The paper's own cache input (Sec. "Neural Incident Radiance Cache": the list of encodings,
 * the amortised surface encoding and the inference-pipeline figure, whose neural input vector
 * has 24 + 25 + (3 + 8 + 4) = 64 entries):
 *   - inputs 0..23: a multiresolution hash grid on x (Mueller et al., "Instant neural graphics
 *     primitives with a multiresolution hash encoding", SIGGRAPH 2022) with 12 levels of 2
 *     trainable FP32 features, input 2 l + f.  Level l has resolution N_l = floor(base_res *
 *     growth^l); x, clamped to the unit cube, is scaled by N_l and the 8 corners of its cell are
 *     blended trilinearly.  A level whose (N_l + 1)^3 vertices fit in T = 2^log2_table entries
 *     is a dense table (vertex v at v0 + (N_l+1) (v1 + (N_l+1) v2)); the others hold T entries
 *     addressed by (v0 * 1 xor v1 * 2654435761 xor v2 * 805459861) mod T;
 *   - inputs 24..48: the real spherical harmonics of degree <= 4 of w (index 24 + l^2 + l + m;
 *     m > 0: sqrt(2) K cos(m phi) P_l^m, m < 0: sqrt(2) K sin(|m| phi) P_l^|m|, no
 *     Condon-Shortley phase; w is taken as unit length);
 *   - inputs 49..63: the surface values phi: normal (identity), roughness as an 8-bin one-blob
 *     (Mueller et al., "Neural importance sampling", TOG 2019: exp(-(8 r - i - 1/2)^2 / 2) for
 *     bin i), albedo (identity, 1 1 1 for the white Lambertian surface) and a zero slot.
 * Network: 64 -> 4 hidden ReLU layers of width 64 -> 3 -> exp, no biases.  Canonical parameter
 * vector (FP32): W1 [64 x 64], W2, W3, W4 [64 x 64], W5 [3 x 64] (16,576 values), then the grid
 * features [entries][2] with the levels in order.  The grid and the MLP use one Adam state.
 * Supported: width 64, precision NIRC_FP32, NIRC_BF16 or NIRC_FP16 (the layer products; grid
 * features and their interpolation stay FP32 in every precision), for inference, estimation and
 * training alike, loss NIRC_LOSS_REL_L2 or NIRC_LOSS_L2, output NIRC_OUTPUT_RADIANCE; anything
 * else is NIRC_ERR_UNSUPPORTED.  Conventions as above.
 * ========================================================================================== */
typedef struct nirc_hash_model nirc_hash_model;

/* Grid shape (host).  log2_table 10..22 (18: 2,334,718 entries, 18.7 MB of FP32 features with
 * base_res 16 and growth 1.5), base_res >= 2, growth in [1, 4], N_11 <= 2^20. */
typedef struct {
    int32_t log2_table;
    int32_t base_res;
    float growth;
} nirc_hash_grid;

/* Entries of the grid (0 for an invalid grid). */
int64_t nirc_hash_entries(const nirc_hash_grid *grid);

/* Length of the canonical parameter vector: 16,576 + 2 * entries (0 for an invalid grid). */
int64_t nirc_hash_n_params(const nirc_hash_grid *grid);

/* Resolution, first entry and dense flag (1/0) of the 12 levels, host arrays of 12. */
nirc_status nirc_hash_levels(const nirc_hash_grid *grid, int32_t *res, int64_t *offset, int32_t *dense);

/* Bytes of model state (FP32 parameters, Adam moments, packed layers in the model's precision,
 * step, flags) and of training workspace for batches up to max_batch (0 for an invalid
 * configuration). */
size_t nirc_hash_state_bytes(const nirc_config *cfg, const nirc_hash_grid *grid);
size_t nirc_hash_workspace_bytes(const nirc_config *cfg, const nirc_hash_grid *grid, int64_t max_batch);

/* Creates a model on caller memory (state: 256-byte aligned, nirc_hash_state_bytes; workspace:
 * NULL for inference only, else 256-byte aligned) from init_w [nirc_hash_n_params] (device). */
nirc_status nirc_hash_create(const nirc_config *cfg, const nirc_hash_grid *grid, void *state, size_t state_bytes,
                             void *workspace, size_t workspace_bytes, const float *init_w, void *stream,
                             nirc_hash_model **out);
nirc_status nirc_hash_destroy(nirc_hash_model *model);

/* Replace (and reset Adam) / read the canonical parameter vector [nirc_hash_n_params]. */
nirc_status nirc_hash_set_weights(nirc_hash_model *model, const float *w, void *stream);
nirc_status nirc_hash_get_weights(const nirc_hash_model *model, float *w, void *stream);

/* Checkpoint / resume: the whole training state (parameters, Adam moments and step, flags) as
 * one blob of exactly nirc_hash_state_bytes bytes (device memory, 4-byte aligned). */
nirc_status nirc_hash_get_state(const nirc_hash_model *model, void *blob, size_t blob_bytes, void *stream);
nirc_status nirc_hash_set_state(nirc_hash_model *model, const void *blob, size_t blob_bytes, void *stream);

/* Cache predictions for explicit queries: rgb [queries.count][3]. */
nirc_status nirc_hash_infer(const nirc_hash_model *model, nirc_points points, nirc_queries queries, float *rgb,
                            void *stream);

/* The fused two-level estimator with this cache, as tlmc_estimate (same directions, same
 * residual handling, same outputs); the surface part (grid lookup, phi and its first-layer
 * product) is computed once per point and shared by its N + 1 queries. */
nirc_status nirc_hash_estimate(const nirc_hash_model *model, nirc_points points, const nirc_lobes *field /* host */,
                               int32_t n_cache, uint64_t seed, uint64_t frame, const float *residual_radiance,
                               float *out_tl, float *out_c, float *out_r, void *stream);

/* Loss (device float, may be NULL) and gradient grad [nirc_hash_n_params] (device) of a batch,
 * without an update: MLP weight gradients, and for every grid entry the sum over samples of
 * its trilinear weight times the loss gradient of its level's input (entries no sample
 * touches get 0).  Needs the workspace. */
nirc_status nirc_hash_loss_grad(nirc_hash_model *model, nirc_points points, nirc_queries queries,
                                const float *target, float *grad, float *loss, void *stream);

/* One Adam step over the whole parameter vector with the given gradient (skipped, with
 * NIRC_FLAG_NONFINITE_GRAD raised, when it holds a non-finite value). */
nirc_status nirc_hash_adam_step(nirc_hash_model *model, const float *grad, void *stream);

/* Loss and gradient into the workspace, then the Adam step. */
nirc_status nirc_hash_train_step(nirc_hash_model *model, nirc_points points, nirc_queries queries,
                                 const float *target, float *loss, void *stream);

/* One frame's online training, as nirc_train_frame: steps x (tlmc_train_batch, then
 * nirc_hash_train_step) with the samples in the workspace (nirc_hash_workspace_bytes of at least
 * `batch`); loss (device float, may be NULL) receives the last step's loss. */
nirc_status nirc_hash_train_frame(nirc_hash_model *model, nirc_points points, const nirc_lobes *field /* host */,
                                  int64_t batch, int32_t steps, uint64_t seed, uint64_t frame, float *loss,
                                  void *stream);

/* Flags raised by training (synchronises the stream); 0xFFFFFFFF on error. */
uint32_t nirc_hash_read_flags(const nirc_hash_model *model, void *stream);

/* Matrix-core microbenchmark (measurement, not part of the method): `blocks` workgroups of 256
 * threads, each wave running `iters` (a multiple of 32) iterations of 8 independent MFMA accumulations
 * (16x16x32 for NIRC_BF16 / NIRC_FP16: 16,384 FLOPs each; 16x16x4 FP32 for NIRC_FP32: 2,048
 * FLOPs each) followed by `fmas` (0, 32 or 64) independent FP32 FMAs per lane.  Writes one float
 * per thread to sink [blocks x 256] (device) so that nothing is optimised away.  Timed by the
 * caller: 8 x iters x 4 x blocks MFMAs per launch give the matrix rate the roofline fractions
 * are also quoted against (beside the vendor peak); fmas > 0 shows whether FP32 VALU work hides
 * under the MFMAs.  NIRC_ERR_INVALID_ARG for other precisions, counts or a NULL sink. */
nirc_status nirc_probe_mfma(int32_t precision, int32_t iters, int32_t fmas, int32_t blocks, float *sink,
                            void *stream);

/* Atomics microbenchmark (measurement, not part of the method): `blocks` workgroups of 256
 * threads; thread t adds 1 to element e(i) of buf for i = t + r * T, r < reps (T threads), where
 * lanes_per_line (1, 2, 4, 8 or 16) consecutive i share one 128-byte line (16 elements) and
 * consecutive groups take consecutive lines, wrapping at buf's end (buf_elems a power of two,
 * >= 16; device).  64-bit integer adds without return, as the hash-grid gradient scatter makes:
 * T x reps adds per launch, timed by the caller.  NIRC_ERR_INVALID_ARG on other values. */
nirc_status nirc_probe_atomics(int32_t lanes_per_line, int32_t reps, int32_t blocks, uint64_t *buf, int64_t buf_elems,
                               void *stream);

const char *nirc_status_string(nirc_status s);

#ifdef __cplusplus
}
#endif

#endif /* NIRC_H */
