// C ABI of the NIRC library: argument validation, state/workspace layout and kernel launches.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <new>
#include <string.h>

#include "nirc_h16.hpp"

using namespace nirc;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

bool width_ok(int32_t w) { return w == 64 || w == 128; }

// State layout (each piece 256-byte aligned): master | m | v | packed FP32 | packed 16-bit (BF16
// and FP16 models only) | step | flags | bad | loss scale (FP32), good-step count and the Adam
// kernel's finished-workgroup count (uint32, zero between steps).
struct StateLayout {
    size_t master, m, v, packed, packed16, step, flags, bad, scale, total;
    StateLayout(int W, int prec) {
        const size_t np = (size_t)n_params(W) * sizeof(float);
        size_t o = 0;
        master = o; o += align_up(np);
        m = o; o += align_up(np);
        v = o; o += align_up(np);
        packed = o; o += align_up((size_t)F32Layout{W}.total() * sizeof(float));
        packed16 = o;
        if (prec != NIRC_FP32) o += align_up((size_t)H16Layout{W}.total() * sizeof(uint16_t));
        step = o; o += align_up(sizeof(int64_t));
        flags = o; o += align_up(sizeof(uint32_t));
        bad = o; o += align_up(sizeof(uint32_t));
        scale = o; o += align_up(3 * sizeof(uint32_t));
        total = o;
    }
};

// Workspace layout: partials [nblocks][np] | loss partials [nblocks] | grad [np] | loss |
// residual-variance loss pre-pass (predictions [B][3], kFrBlocks x 3 FP32 partials, F_r [3]; only
// for NIRC_LOSS_VAR) | training samples of nirc_train_frame (point [B], wx, wy, wz [B],
// target [B][3]).
struct WorkLayout {
    size_t partials, loss_partials, grad, loss, pred, fr_part, fr, samples, total;
    WorkLayout(int W, int nblocks, int64_t var_batch = 0, int64_t sample_batch = 0) {
        const size_t np = (size_t)n_params(W);
        size_t o = 0;
        partials = o; o += align_up((size_t)nblocks * np * sizeof(float));
        loss_partials = o; o += align_up((size_t)nblocks * sizeof(float));
        grad = o; o += align_up(np * sizeof(float));
        loss = o; o += align_up(sizeof(float));
        pred = o; o += var_batch ? align_up((size_t)var_batch * 3 * sizeof(float)) : 0;
        fr_part = o; o += var_batch ? align_up((size_t)kFrBlocks * 3 * sizeof(float)) : 0;
        fr = o; o += var_batch ? align_up(4 * sizeof(float)) : 0;
        samples = o; o += align_up((size_t)kFrameSampleSteps * sample_batch * 7 * sizeof(float));
        total = o;
    }
};

int64_t var_rows(const nirc_config &cfg, int64_t batch) { return cfg.loss == NIRC_LOSS_VAR ? batch : 0; }

// Gradient-partial slabs of a batch: the grid of the precision's gradient kernel.  Every
// workspace layout of a model (sizing, the partials, the reduced gradient after them) takes its
// count from here, so that the layouts agree whatever the kernels' rounds are.
int grad_blocks(int32_t precision, int64_t batch) {
    return precision != NIRC_FP32 ? train_blocks16(batch) : train_blocks(batch);
}

nirc_status check_points(const nirc_points &p) {
    if (p.count < 0 || p.count > INT32_MAX) return NIRC_ERR_INVALID_ARG;
    if (p.count > 0 && (!p.px || !p.py || !p.pz || !p.nx || !p.ny || !p.nz || !p.rough))
        return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

nirc_status check_queries(const nirc_queries &q, const nirc_points &p) {
    if (q.count < 0) return NIRC_ERR_INVALID_ARG;
    if (q.count > 0 && (!q.wx || !q.wy || !q.wz)) return NIRC_ERR_INVALID_ARG;
    if (q.count > 0 && p.count == 0) return NIRC_ERR_INVALID_ARG;
    if (!q.point && q.count > p.count) return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

Points to_points(const nirc_points &p) { return Points{p.px, p.py, p.pz, p.nx, p.ny, p.nz, p.rough, p.count}; }
// err: where a point index out of range is reported (the model's sticky flags, or the step's
// flags of a training step, which then skips its update)
Queries to_queries(const nirc_queries &q, uint32_t *err) { return Queries{q.wx, q.wy, q.wz, q.point, q.count, err}; }

nirc_status hip_status(hipError_t e) { return e == hipSuccess ? NIRC_OK : NIRC_ERR_HIP; }

}  // namespace

struct nirc_model {
    nirc_config cfg;
    int W;
    int64_t np;
    float *master, *m, *v, *packed;
    uint16_t *packed16;   // NULL for FP32 models
    int64_t *step;
    uint32_t *flags, *bad;
    float *scale;          // the current loss scale (dynamic for FP16 models)
    uint32_t *good;        // finite steps since the scale last changed
    uint32_t *done;        // finished workgroups of the running Adam launch (zero between steps)
    char *ws;
    size_t ws_bytes;
    // FP16 models scale their loss dynamically; BF16 and FP32 keep cfg.loss_scale
    float *dyn() const { return cfg.precision == NIRC_FP16 ? scale : nullptr; }
    uint32_t *dyn_good() const { return cfg.precision == NIRC_FP16 ? good : nullptr; }
};

extern "C" {

const char *nirc_status_string(nirc_status s) {
    switch (s) {
    case NIRC_OK: return "ok";
    case NIRC_ERR_INVALID_ARG: return "invalid argument";
    case NIRC_ERR_UNSUPPORTED: return "unsupported configuration";
    case NIRC_ERR_WORKSPACE: return "state or workspace buffer too small";
    case NIRC_ERR_HIP: return "HIP error";
    default: return "unknown status";
    }
}

int64_t nirc_n_params(int32_t width) { return width_ok(width) ? n_params(width) : 0; }

static nirc_status check_config(const nirc_config *cfg) {
    if (!cfg) return NIRC_ERR_INVALID_ARG;
    if (!width_ok(cfg->width)) return NIRC_ERR_UNSUPPORTED;
    if (cfg->loss != NIRC_LOSS_REL_L2 && cfg->loss != NIRC_LOSS_L2 && cfg->loss != NIRC_LOSS_VAR)
        return NIRC_ERR_INVALID_ARG;
    if (cfg->output != NIRC_OUTPUT_RADIANCE && cfg->output != NIRC_OUTPUT_VISIBILITY &&
        cfg->output != NIRC_OUTPUT_RADIANCE_OCCLUDED)
        return NIRC_ERR_INVALID_ARG;
    if (cfg->precision != NIRC_FP32 && cfg->precision != NIRC_BF16 && cfg->precision != NIRC_FP16)
        return NIRC_ERR_UNSUPPORTED;
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->adam_eps > 0.0f) ||
        !(cfg->loss_eps > 0.0f) || !(cfg->loss_scale > 0.0f))
        return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

size_t nirc_state_bytes(const nirc_config *cfg) {
    if (check_config(cfg) != NIRC_OK) return 0;
    return StateLayout(cfg->width, cfg->precision).total;
}

size_t nirc_workspace_bytes(const nirc_config *cfg, int64_t max_batch) {
    if (check_config(cfg) != NIRC_OK || max_batch < 0) return 0;
    return WorkLayout(cfg->width, grad_blocks(cfg->precision, max_batch), var_rows(*cfg, max_batch), max_batch).total;
}

nirc_status nirc_create(const nirc_config *cfg, void *state, size_t state_bytes, void *workspace,
                        size_t workspace_bytes, const float *init_w, void *stream, nirc_model **out) {
    nirc_status st = check_config(cfg);
    if (st != NIRC_OK) return st;
    if (!state || !init_w || !out || ((uintptr_t)state % kAlign) != 0) return NIRC_ERR_INVALID_ARG;
    if (workspace && ((uintptr_t)workspace % kAlign) != 0) return NIRC_ERR_INVALID_ARG;
    const StateLayout sl(cfg->width, cfg->precision);
    if (state_bytes < sl.total) return NIRC_ERR_WORKSPACE;
    nirc_model *m = new (std::nothrow) nirc_model;
    if (!m) return NIRC_ERR_INVALID_ARG;
    char *base = (char *)state;
    m->cfg = *cfg;
    m->W = cfg->width;
    m->np = n_params(m->W);
    m->master = (float *)(base + sl.master);
    m->m = (float *)(base + sl.m);
    m->v = (float *)(base + sl.v);
    m->packed = (float *)(base + sl.packed);
    m->packed16 = cfg->precision != NIRC_FP32 ? (uint16_t *)(base + sl.packed16) : nullptr;
    m->step = (int64_t *)(base + sl.step);
    m->flags = (uint32_t *)(base + sl.flags);
    m->bad = (uint32_t *)(base + sl.bad);
    m->scale = (float *)(base + sl.scale);
    m->good = (uint32_t *)(base + sl.scale + sizeof(float));
    m->done = (uint32_t *)(base + sl.scale + sizeof(float) + sizeof(uint32_t));
    m->ws = (char *)workspace;
    m->ws_bytes = workspace ? workspace_bytes : 0;
    st = nirc_set_weights(m, init_w, stream);
    if (st == NIRC_OK) {
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = launch_fill_u32(m->flags, 1, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(m->bad, 1, 0u, s);
        st = hip_status(e);
    }
    if (st != NIRC_OK) {
        delete m;
        return st;
    }
    *out = m;
    return NIRC_OK;
}

nirc_status nirc_destroy(nirc_model *model) {
    delete model;
    return NIRC_OK;
}

nirc_status nirc_set_weights(nirc_model *model, const float *w, void *stream) {
    if (!model || !w) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_copy_f32(model->master, w, model->np, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->m, model->np, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->v, model->np, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->step, 2, 0u, s);
    // the loss scale starts again from the configured one
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->scale, 1, __builtin_bit_cast(uint32_t, model->cfg.loss_scale), s);
    if (e == hipSuccess) e = launch_fill_u32(model->good, 2, 0u, s);   // good-step and workgroup counts
    if (e == hipSuccess) e = launch_pack(model->packed, model->master, model->W, s);
    if (e == hipSuccess && model->packed16)
        e = launch_pack16(model->packed16, model->master, model->W, model->cfg.precision, s);
    return hip_status(e);
}

nirc_status nirc_get_weights(const nirc_model *model, float *w, void *stream) {
    if (!model || !w) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_copy_f32(w, model->master, model->np, (hipStream_t)stream));
}

// The state is one region from the FP32 weights on (StateLayout); a blob is its image.
nirc_status nirc_get_state(const nirc_model *model, void *blob, size_t blob_bytes, void *stream) {
    if (!model || !blob || ((uintptr_t)blob % 4) != 0) return NIRC_ERR_INVALID_ARG;
    const size_t bytes = StateLayout(model->W, model->cfg.precision).total;
    if (blob_bytes != bytes) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_copy_f32((float *)blob, model->master, (int64_t)(bytes / 4), (hipStream_t)stream));
}

nirc_status nirc_set_state(nirc_model *model, const void *blob, size_t blob_bytes, void *stream) {
    if (!model || !blob || ((uintptr_t)blob % 4) != 0) return NIRC_ERR_INVALID_ARG;
    const size_t bytes = StateLayout(model->W, model->cfg.precision).total;
    if (blob_bytes != bytes) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_copy_f32(model->master, (const float *)blob, (int64_t)(bytes / 4), s);
    // the packed copies follow the restored FP32 weights whatever precision wrote the blob
    if (e == hipSuccess) e = launch_pack(model->packed, model->master, model->W, s);
    if (e == hipSuccess && model->packed16)
        e = launch_pack16(model->packed16, model->master, model->W, model->cfg.precision, s);
    return hip_status(e);
}

nirc_status nirc_get_adam(const nirc_model *model, float *m, float *v, int64_t *step, void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipSuccess;
    if (m) e = launch_copy_f32(m, model->m, model->np, s);
    if (e == hipSuccess && v) e = launch_copy_f32(v, model->v, model->np, s);
    if (e == hipSuccess && step) e = launch_copy_f32((float *)step, (const float *)model->step, 2, s);
    return hip_status(e);
}

uint32_t nirc_read_flags(const nirc_model *model, void *stream) {
    if (!model) return 0xFFFFFFFFu;
    uint32_t f = 0;
    if (hipMemcpyAsync(&f, model->flags, sizeof(f), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return 0xFFFFFFFFu;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return 0xFFFFFFFFu;
    return f;
}

float nirc_read_loss_scale(const nirc_model *model, void *stream) {
    if (!model) return -1.0f;
    float f = 0.0f;
    if (hipMemcpyAsync(&f, model->scale, sizeof(f), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return -1.0f;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return -1.0f;
    return f;
}

nirc_status nirc_clear_flags(nirc_model *model, void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_fill_u32(model->flags, 1, 0u, (hipStream_t)stream));
}

nirc_status nirc_encode(nirc_points points, nirc_queries queries, float *features, void *stream) {
    nirc_status st = check_points(points);
    if (st == NIRC_OK) st = check_queries(queries, points);
    if (st != NIRC_OK) return st;
    if (queries.count > 0 && !features) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_encode(to_points(points), to_queries(queries, nullptr), features, (hipStream_t)stream));
}

nirc_status nirc_infer(const nirc_model *model, nirc_points points, nirc_queries queries, float *rgb,
                       void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st == NIRC_OK) st = check_queries(queries, points);
    if (st != NIRC_OK) return st;
    if (queries.count > 0 && !rgb) return NIRC_ERR_INVALID_ARG;
    const void *pk = model->packed16 ? (const void *)model->packed16 : (const void *)model->packed;
    return hip_status(launch_infer(model->W, model->cfg.precision, to_points(points), to_queries(queries, model->flags), pk, rgb,
                                   model->cfg.output == NIRC_OUTPUT_VISIBILITY,
                                   (hipStream_t)stream));
}

nirc_status tlmc_sample_dirs(nirc_points points, int32_t n_cache, uint64_t seed, uint64_t frame,
                             float *dirs, void *stream) {
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (n_cache < 1 || n_cache > 4096 || (points.count > 0 && !dirs)) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_sample_dirs(to_points(points), n_cache, seed, frame, dirs, (hipStream_t)stream));
}

nirc_status tlmc_estimate(const nirc_model *model, nirc_points points, const nirc_lobes *field,
                          int32_t n_cache, uint64_t seed, uint64_t frame, const float *residual_radiance,
                          float *out_tl, float *out_c, float *out_r, void *stream) {
    if (!model || (!field && !residual_radiance)) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (n_cache < 1 || n_cache > 4096 || (points.count > 0 && !out_tl)) return NIRC_ERR_INVALID_ARG;
    const void *pk = model->packed16 ? (const void *)model->packed16 : (const void *)model->packed;
    nirc_lobes none;
    memset(&none, 0, sizeof(none));
    return hip_status(launch_tlmc(model->W, model->cfg.precision, to_points(points), field ? *field : none, pk,
                                  n_cache, seed, frame, model->cfg.output, residual_radiance, out_tl, out_c, out_r,
                                  (hipStream_t)stream));
}

nirc_status tlmc_estimate_biased(const nirc_model *model, nirc_points points, const nirc_lobes *field,
                                 int32_t n_cache, uint64_t seed, uint64_t frame, const float *residual_radiance,
                                 float *out_b, float *out_c, int32_t *out_continue, void *stream) {
    if (points.count > 0 && (!out_b || !out_c)) return NIRC_ERR_INVALID_ARG;
    // F_c (and F_tl, overwritten below) by the fused estimator, then the per-point decision
    nirc_status st = tlmc_estimate(model, points, field, n_cache, seed, frame, residual_radiance, out_b, out_c,
                                   nullptr, stream);
    if (st != NIRC_OK || points.count == 0) return st;
    nirc_lobes none;
    memset(&none, 0, sizeof(none));
    return hip_status(launch_bth(to_points(points), field ? *field : none, n_cache, seed, frame, model->cfg.output,
                                 residual_radiance, out_c, out_b, out_continue, (hipStream_t)stream));
}

static bool output_ok(int32_t o) {
    return o == NIRC_OUTPUT_RADIANCE || o == NIRC_OUTPUT_VISIBILITY || o == NIRC_OUTPUT_RADIANCE_OCCLUDED;
}

nirc_status tlmc_train_batch(nirc_points points, const nirc_lobes *field, int64_t batch, uint64_t seed,
                             uint64_t frame, uint32_t step, int32_t output, int32_t *point, float *wx, float *wy,
                             float *wz, float *target, void *stream) {
    if (!field || batch < 0 || batch > INT32_MAX || !output_ok(output)) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (batch > 0 && (points.count == 0 || !point || !wx || !wy || !wz || !target)) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_train_batch(to_points(points), *field, batch, seed, frame, step, output, point, wx, wy,
                                         wz, target, (hipStream_t)stream));
}

// Gauss-Legendre nodes and weights on [0, 1] (Newton's method on the Legendre recurrence).
static void gauss_legendre01(int n, QuadNodes &q) {
    q.n = n;
    for (int i = 0; i < n; ++i) {
        double t = std::cos(3.14159265358979323846 * (i + 0.75) / (n + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = t;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (t * p1 - p0) / (t * t - 1.0);
            const double dt = p1 / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-15) break;
        }
        q.x[i] = 0.5 * (1.0 - t);
        q.w[i] = 1.0 / ((1.0 - t * t) * dp * dp);
    }
}

nirc_status tlmc_reference_occluded(nirc_points points, const nirc_lobes *field, int32_t n_nodes, double *F,
                                    void *stream) {
    if (!field || n_nodes < 8 || n_nodes > kMaxQuadNodes) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (points.count > 0 && !F) return NIRC_ERR_INVALID_ARG;
    QuadNodes q;
    gauss_legendre01(n_nodes, q);
    return hip_status(launch_reference_occluded(to_points(points), *field, q, F, (hipStream_t)stream));
}

// Gradient partials + reduction into `grad`/`loss`; the step's `bad` flag is raised on a
// non-finite value.
static nirc_status grad_into(nirc_model *model, const nirc_points &points, const nirc_queries &queries,
                             const float *target, const float *d_rgb, float *grad, float *loss, uint32_t *err,
                             char *ws, size_t ws_bytes, hipStream_t s) {
    nirc_status st = check_points(points);
    if (st == NIRC_OK) st = check_queries(queries, points);
    if (st != NIRC_OK) return st;
    if (queries.count < 1 || !grad) return NIRC_ERR_INVALID_ARG;
    const bool h16 = model->packed16 != nullptr;
    const int nb = grad_blocks(model->cfg.precision, queries.count);
    const bool var = target && model->cfg.loss == NIRC_LOSS_VAR;
    const WorkLayout wl(model->W, nb, var ? queries.count : 0);
    if (!ws || ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    float *partials = (float *)(ws + wl.partials);
    float *lpart = (float *)(ws + wl.loss_partials);
    // 16-bit models: the batch size is folded into the loss scale, so that per-sample deltas stay
    // near unit magnitude in the 16-bit operands; the reduction divides it out again
    const float scale = h16 ? model->cfg.loss_scale * (float)queries.count : model->cfg.loss_scale;
    TrainArgs a{target, d_rgb, model->cfg.loss_eps, scale, model->cfg.loss, nullptr,
                model->cfg.output == NIRC_OUTPUT_VISIBILITY, model->dyn()};
    if (var) {   // the residual-variance loss needs F_r = mean(t - y) of this batch first
        float *pred = (float *)(ws + wl.pred);
        float *fr = (float *)(ws + wl.fr);
        const void *pk = h16 ? (const void *)model->packed16 : (const void *)model->packed;
        hipError_t e = launch_infer(model->W, model->cfg.precision, to_points(points), to_queries(queries, err), pk, pred,
                                    model->cfg.output == NIRC_OUTPUT_VISIBILITY, s);
        if (e == hipSuccess)
            e = launch_residual_mean(pred, target, queries.count, (float *)(ws + wl.fr_part), fr, s);
        if (e != hipSuccess) return NIRC_ERR_HIP;
        a.fr = fr;
    }
    hipError_t e = h16 ? launch_grad_partials16(model->W, model->cfg.precision, to_points(points),
                                                to_queries(queries, err), model->packed16, a, partials, lpart, nb, s)
                       : launch_grad_partials(model->W, to_points(points), to_queries(queries, err), model->packed, a,
                                              partials, lpart, nb, s);
    if (e != hipSuccess) return NIRC_ERR_HIP;
    const float loss_norm = 1.0f / (3.0f * (float)queries.count);
    e = launch_reduce_grad(model->W, partials, lpart, nb, 1.0f / scale, loss_norm, grad, loss, model->bad, s,
                           model->dyn(), (float)queries.count);
    return hip_status(e);
}

nirc_status nirc_loss_grad(nirc_model *model, nirc_points points, nirc_queries queries, const float *target,
                           float *grad, float *loss, void *stream) {
    if (!model || !target) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    nirc_status st = grad_into(model, points, queries, target, nullptr, grad, loss, model->flags, model->ws, model->ws_bytes, s);
    if (st != NIRC_OK) return st;
    // a standalone gradient does not start a step: clear the step's flag again
    return hip_status(launch_fill_u32(model->bad, 1, 0u, s));
}

nirc_status nirc_backward(nirc_model *model, nirc_points points, nirc_queries queries, const float *d_rgb,
                          float *grad, void *stream) {
    if (!model || !d_rgb) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    nirc_status st = grad_into(model, points, queries, nullptr, d_rgb, grad, nullptr, model->flags, model->ws, model->ws_bytes, s);
    if (st != NIRC_OK) return st;
    return hip_status(launch_fill_u32(model->bad, 1, 0u, s));
}

nirc_status nirc_adam_step(nirc_model *model, const float *grad, void *stream) {
    if (!model || !grad) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_check_finite(model->W, grad, model->bad, s);
    if (e == hipSuccess)
        e = launch_adam(model->W, model->master, model->m, model->v, grad, model->step, model->flags, model->bad,
                        model->cfg.lr, model->cfg.beta1, model->cfg.beta2, model->cfg.adam_eps, model->packed,
                        model->packed16, model->cfg.precision, s, model->done);
    return hip_status(e);
}

// Gradient into the workspace `ws`, then Adam on it.
static nirc_status train_step_on(nirc_model *model, const nirc_points &points, const nirc_queries &queries,
                                 const float *target, float *loss, char *ws, size_t ws_bytes, hipStream_t s) {
    if (!model || !target) return NIRC_ERR_INVALID_ARG;
    const WorkLayout wl(model->W, grad_blocks(model->cfg.precision, queries.count));
    if (!ws || ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    float *grad = (float *)(ws + wl.grad);
    float *wloss = (float *)(ws + wl.loss);
    nirc_status st =
        grad_into(model, points, queries, target, nullptr, grad, loss ? loss : wloss, model->bad, ws, ws_bytes, s);
    if (st != NIRC_OK) return st;
    hipError_t e = launch_adam(model->W, model->master, model->m, model->v, grad, model->step, model->flags,
                               model->bad, model->cfg.lr, model->cfg.beta1, model->cfg.beta2, model->cfg.adam_eps,
                               model->packed, model->packed16, model->cfg.precision, s, model->done, model->dyn(),
                               model->dyn_good());
    return hip_status(e);
}

nirc_status nirc_train_step(nirc_model *model, nirc_points points, nirc_queries queries, const float *target,
                            float *loss, void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    return train_step_on(model, points, queries, target, loss, model->ws, model->ws_bytes, (hipStream_t)stream);
}

// ------------------------------------------------------------------------------------------
// Training step without workspace: the gradient partials, reduced gradient and loss of one step
// live in a static device array of the library.  Sized for NIRC_STATIC_MAX_BATCH samples at
// width 128 (the larger layout): at most 32 partial slabs of 70,016 floats, the gradient, the
// loss and the residual-variance pre-pass.  Each GPU holds its own copy at its own address;
// host code reaches it only through the address hipGetSymbolAddress returns on that device.
namespace {
constexpr size_t cx_align(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
constexpr int64_t kStaticSlabs = (NIRC_STATIC_MAX_BATCH + 63) / 64;
constexpr size_t kStaticNp = 128 * 160 + 3 * 128 * 128 + 3 * 128;
constexpr size_t kScratchBytes = cx_align(kStaticSlabs * kStaticNp * sizeof(float)) +
                                 cx_align(kStaticSlabs * sizeof(float)) + cx_align(kStaticNp * sizeof(float)) +
                                 cx_align(sizeof(float)) + cx_align((size_t)NIRC_STATIC_MAX_BATCH * 3 * sizeof(float)) +
                                 cx_align((size_t)kFrBlocks * 3 * sizeof(float)) + cx_align(4 * sizeof(float));
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char *g_scratch_ptr[kMaxDevices];   // per device, set once with that device current
}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

// The device address of this GPU's `scratch` (looked up once per device); NULL on failure.
static char *scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
        g_scratch_ptr[dev] = (char *)p;
    }
    return g_scratch_ptr[dev];
}

nirc_status nirc_train_step_static(nirc_model *model, nirc_points points, nirc_queries queries, const float *target,
                                   float *loss, void *stream) {
    if (!model || queries.count > NIRC_STATIC_MAX_BATCH) return NIRC_ERR_INVALID_ARG;
    const WorkLayout wl(model->W, grad_blocks(model->cfg.precision, queries.count),
                        var_rows(model->cfg, queries.count));
    if (wl.total > kScratchBytes) return NIRC_ERR_INVALID_ARG;   // not reached for valid configurations
    char *ws = scratch_on_current_device();
    if (!ws) return NIRC_ERR_HIP;
    // every part of the layout is written before it is read within the step: nothing to clear
    return train_step_on(model, points, queries, target, loss, ws, kScratchBytes, (hipStream_t)stream);
}

nirc_status nirc_train_frame(nirc_model *model, nirc_points points, const nirc_lobes *field, int64_t batch,
                             int32_t steps, uint64_t seed, uint64_t frame, float *loss, void *stream) {
    if (!model || !field || batch < 1 || batch > INT32_MAX || steps < 0) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK || points.count < 1) return NIRC_ERR_INVALID_ARG;
    const WorkLayout wl(model->W, grad_blocks(model->cfg.precision, batch), var_rows(model->cfg, batch), batch);
    if (!model->ws || model->ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    // the samples of up to kFrameSampleSteps steps in one launch (they do not depend on the
    // weights), 7 values per sample and step: point, wx, wy, wz, target x 3
    const int64_t stride = 7 * batch;
    for (int32_t k = 0; k < steps; ++k) {
        float *smp = (float *)(model->ws + wl.samples) + (k % kFrameSampleSteps) * stride;
        int32_t *pidx = (int32_t *)smp;
        float *wx = smp + batch, *wy = wx + batch, *wz = wy + batch, *tgt = wz + batch;
        if (k % kFrameSampleSteps == 0) {
            const hipError_t e = launch_train_batch(to_points(points), *field, batch, seed, frame, (uint32_t)k,
                                                    model->cfg.output, pidx, wx, wy, wz, tgt, s,
                                                    std::min(kFrameSampleSteps, steps - k), stride);
            if (e != hipSuccess) return NIRC_ERR_HIP;
        }
        nirc_queries q{wx, wy, wz, pidx, batch};
        st = nirc_train_step(model, points, q, tgt, k + 1 == steps ? loss : nullptr, s);
        if (st != NIRC_OK) return st;
    }
    return NIRC_OK;
}

size_t tlmc_batch_bytes(void) { return sizeof(BatchDesc); }

nirc_status tlmc_batch_build(const tlmc_request *requests, int32_t n, void *list) {
    if (!requests || !list || n < 1 || n > TLMC_BATCH_MAX_REQUESTS || n > kBatchMaxRequests)
        return NIRC_ERR_INVALID_ARG;
    BatchDesc *d = (BatchDesc *)list;
    memset(d, 0, sizeof(*d));
    const nirc_model *m0 = requests[0].model;
    if (!m0) return NIRC_ERR_INVALID_ARG;
    if (m0->W != 64) return NIRC_ERR_UNSUPPORTED;
    int64_t chunk = 0;
    for (int i = 0; i < n; ++i) {
        const tlmc_request &r = requests[i];
        if (!r.model || r.model->W != m0->W || r.model->cfg.precision != m0->cfg.precision ||
            r.model->cfg.output != m0->cfg.output)
            return NIRC_ERR_INVALID_ARG;
        if (check_points(r.points) != NIRC_OK || r.points.count < 1) return NIRC_ERR_INVALID_ARG;
        if (r.n_cache < 1 || r.n_cache > 4096 || !r.out_tl) return NIRC_ERR_INVALID_ARG;
        BatchRequest &q = d->req[i];
        q.pts = to_points(r.points);
        q.packed = r.model->packed16 ? (const void *)r.model->packed16 : (const void *)r.model->packed;
        q.lobes = r.field;
        q.n_cache = r.n_cache;
        q.dn = make_divn(r.n_cache);
        q.key0 = (uint32_t)r.seed;
        q.key1 = (uint32_t)(r.seed >> 32);
        q.frame = (uint32_t)r.frame;
        q.rrad = r.residual_radiance;
        q.mode = r.model->cfg.output;
        q.out_tl = r.out_tl;
        q.out_c = r.out_c;
        q.out_r = r.out_r;
        q.chunk_begin = (int32_t)chunk;
        const int64_t groups = (r.points.count + 15) / 16;
        chunk += (groups + kBatchChunkGroups - 1) / kBatchChunkGroups;
        if (chunk > INT32_MAX) return NIRC_ERR_INVALID_ARG;
    }
    d->n_requests = n;
    d->total_chunks = (int32_t)chunk;
    d->width = m0->W;
    d->precision = m0->cfg.precision;
    return NIRC_OK;
}

nirc_status tlmc_estimate_batch(const void *list, int32_t width, int32_t precision, int32_t output, void *stream) {
    if (!list) return NIRC_ERR_INVALID_ARG;
    if (width != 64) return NIRC_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    const int grid = kMaxResidentBlocks;   // one persistent workgroup per CU
    if (!output_ok(output)) return NIRC_ERR_INVALID_ARG;
    if (precision == NIRC_FP32)
        return hip_status(launch_tlmc_multi_f32(width, output, (const BatchDesc *)list, grid, s));
    if (precision == NIRC_BF16 || precision == NIRC_FP16)
        return hip_status(launch_tlmc_multi_h16(width, precision, output, (const BatchDesc *)list, grid, s));
    return NIRC_ERR_INVALID_ARG;
}

size_t tlmc_unfused_workspace_bytes(int64_t points, int32_t n_cache, int32_t stage) {
    if (points < 0 || points > INT32_MAX || n_cache < 1 || n_cache > 4096 || stage < 0 || stage > 3) return 0;
    if (points * (int64_t)(n_cache + 1) > (int64_t)UINT32_MAX) return 0;
    return stage == 3 ? 0 : ablation_workspace_bytes(points, n_cache, stage);
}

nirc_status tlmc_estimate_unfused(const nirc_model *model, nirc_points points, const nirc_lobes *field,
                                  int32_t n_cache, uint64_t seed, uint64_t frame, int32_t stage, void *workspace,
                                  size_t workspace_bytes, float *out_tl, float *out_c, float *out_r, void *stream) {
    if (!model || !field || stage < 0 || stage > 3) return NIRC_ERR_INVALID_ARG;
    if (model->W != 64 || !model->packed16 || model->cfg.output != NIRC_OUTPUT_RADIANCE) return NIRC_ERR_UNSUPPORTED;
    if (stage == 3)
        return tlmc_estimate(model, points, field, n_cache, seed, frame, nullptr, out_tl, out_c, out_r, stream);
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (n_cache < 1 || n_cache > 4096 || (points.count > 0 && !out_tl)) return NIRC_ERR_INVALID_ARG;
    const size_t need = tlmc_unfused_workspace_bytes(points.count, n_cache, stage);
    if (need == 0 && points.count > 0) return NIRC_ERR_INVALID_ARG;
    if (points.count > 0 && (!workspace || workspace_bytes < need || ((uintptr_t)workspace % kAlign) != 0))
        return NIRC_ERR_WORKSPACE;
    return hip_status(launch_ablation(model->cfg.precision, stage, to_points(points), *field, model->packed16, n_cache,
                                      seed, frame, (char *)workspace, out_tl, out_c, out_r, (hipStream_t)stream));
}

size_t nirc_train_list_bytes(void) { return sizeof(TrainDesc); }

nirc_status nirc_train_list_build(const nirc_train_request *requests, int32_t n, int64_t max_batch, void *list) {
    if (!requests || !list || n < 1 || n > NIRC_TRAIN_BATCH_MAX_REQUESTS || n > kBatchMaxRequests || max_batch < 1 ||
        max_batch > INT32_MAX)
        return NIRC_ERR_INVALID_ARG;
    TrainDesc *d = (TrainDesc *)list;
    memset(d, 0, sizeof(*d));
    const nirc_model *m0 = requests[0].model;
    if (!m0) return NIRC_ERR_INVALID_ARG;
    if (m0->W != 64 || m0->cfg.precision == NIRC_FP32) return NIRC_ERR_UNSUPPORTED;
    int64_t vb = 0;
    for (int i = 0; i < n; ++i) {
        const nirc_train_request &r = requests[i];
        nirc_model *m = r.model;
        if (!m || m->W != m0->W || m->cfg.precision != m0->cfg.precision) return NIRC_ERR_INVALID_ARG;
        if (m->cfg.loss == NIRC_LOSS_VAR) return NIRC_ERR_UNSUPPORTED;
        for (int j = 0; j < i; ++j)
            if (requests[j].model == m) return NIRC_ERR_INVALID_ARG;   // one step of a model at a time
        if (check_points(r.points) != NIRC_OK || r.points.count < 1) return NIRC_ERR_INVALID_ARG;
        if (r.batch < 1 || r.batch > max_batch) return NIRC_ERR_INVALID_ARG;
        const int nb = grad_blocks(m->cfg.precision, r.batch);
        const WorkLayout wl(m->W, nb, 0, r.batch);
        if (!m->ws || m->ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
        TrainReq &t = d->req[i];
        t.pts = to_points(r.points);
        t.lobes = r.field;
        t.packed16 = m->packed16;
        t.master = m->master;
        t.m = m->m;
        t.v = m->v;
        t.step = m->step;
        t.flags = m->flags;
        t.bad = m->bad;
        t.partials = (float *)(m->ws + wl.partials);
        t.lpart = (float *)(m->ws + wl.loss_partials);
        t.grad = (float *)(m->ws + wl.grad);
        t.loss = (float *)(m->ws + wl.loss);
        float *smp = (float *)(m->ws + wl.samples);
        t.sp = (int32_t *)smp;
        t.swx = smp + r.batch;
        t.swy = t.swx + r.batch;
        t.swz = t.swy + r.batch;
        t.stgt = t.swz + r.batch;
        t.batch = r.batch;
        t.key0 = (uint32_t)r.seed;
        t.key1 = (uint32_t)(r.seed >> 32);
        t.frame = (uint32_t)r.frame;
        t.nb = nb;
        t.vb0 = (int32_t)vb;
        vb += nb;
        t.lr = m->cfg.lr;
        t.b1 = m->cfg.beta1;
        t.b2 = m->cfg.beta2;
        t.eps = m->cfg.adam_eps;
        t.loss_eps = m->cfg.loss_eps;
        t.loss_scale = m->cfg.loss_scale;
        t.loss_kind = m->cfg.loss;
        t.output = m->cfg.output;
        t.dyn_scale = m->dyn();
        t.good_steps = m->dyn_good();
        t.done = m->done;
    }
    d->n = n;
    d->total_vb = (int32_t)vb;
    d->width = m0->W;
    d->precision = m0->cfg.precision;
    d->max_batch = max_batch;
    return NIRC_OK;
}

nirc_status nirc_train_frame_batch(const void *list, int32_t steps, int32_t precision, int64_t max_batch,
                                   void *stream) {
    if (!list || steps < 0 || max_batch < 1 || max_batch > INT32_MAX) return NIRC_ERR_INVALID_ARG;
    if (precision != NIRC_BF16 && precision != NIRC_FP16) return NIRC_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    for (int32_t k = 0; k < steps; ++k) {
        const hipError_t e = launch_train_step_multi((const TrainDesc *)list, precision, (uint32_t)k, max_batch, s);
        if (e != hipSuccess) return NIRC_ERR_HIP;
    }
    return NIRC_OK;
}

nirc_status tlmc_reference_table(const nirc_lobes *field, double *table, void *stream) {
    if (!field || !table) return NIRC_ERR_INVALID_ARG;
    for (int j = 0; j < 4; ++j)
        if (!(field->kappa[j] >= 0.0f) || field->kappa[j] > 1000.0f) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_reference_table(*field, table, (hipStream_t)stream));
}

nirc_status tlmc_reference(nirc_points points, const nirc_lobes *field, const double *table, double *F,
                           void *stream) {
    if (!field || !table) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (points.count > 0 && !F) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_reference(to_points(points), *field, table, F, (hipStream_t)stream));
}

size_t tlmc_frame_stats_scratch_bytes(void) { return frame_stats_scratch_bytes(); }

nirc_status tlmc_frame_stats(nirc_points points, const nirc_lobes *field, const double *table, const float *est_tl,
                             const float *est_c, const float *est_r, double eps, void *scratch, double *stats,
                             void *stream) {
    if (!field || !table || !scratch || !stats || !(eps > 0.0)) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points(points);
    if (st != NIRC_OK) return st;
    if (points.count > 0 && !est_tl) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_frame_stats(to_points(points), *field, table, est_tl, est_c, est_r, eps,
                                         (double *)scratch, stats, (hipStream_t)stream));
}

nirc_status tlmc_accumulate(const float *values, int64_t count, double *sum, double *sumsq, void *stream) {
    if (count < 0 || (count > 0 && (!values || !sum || !sumsq))) return NIRC_ERR_INVALID_ARG;
    return hip_status(launch_accumulate(values, count, sum, sumsq, (hipStream_t)stream));
}

}  // extern "C"
