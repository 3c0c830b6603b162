// C ABI of the hash-grid cache input: validation, state/workspace layout and launches.
#include <new>
#include <string.h>

#include "nirc_hash.hpp"

using namespace nirc;

namespace {

constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// State (each piece 256-byte aligned): parameters | m | v | packed layers (16-bit, or FP32 for
// FP32 models) | step | flags | bad.
struct HashState {
    size_t master, m, v, packed16, step, flags, bad, total;
    HashState(int64_t np, int prec) {
        const size_t b = (size_t)np * sizeof(float);
        size_t o = 0;
        master = o; o += align_up(b);
        m = o; o += align_up(b);
        v = o; o += align_up(b);
        packed16 = o;
        o += align_up(prec == NIRC_FP32 ? (size_t)kHash32Packed * sizeof(float) : (size_t)kHashPacked * sizeof(uint16_t));
        step = o; o += align_up(sizeof(int64_t));
        flags = o; o += align_up(sizeof(uint32_t));
        bad = o; o += align_up(sizeof(uint32_t));
        total = o;
    }
};

// Workspace: MLP partials [nblocks][16,576] | loss partials [nblocks] | gradient [np] | loss |
// training samples of nirc_hash_train_frame (point [B], wx, wy, wz [B], target [B][3]).
// Workspace: MLP partials | loss partials | gradient [np] | loss | grid-gradient fixed-point
// accumulators [np - kHashMlp] int64 and their non-finite flag | samples of the frame loop.
struct HashWork {
    size_t partials, loss_partials, grad, loss, gacc, gflag, samples, total;
    HashWork(int64_t np, int nblocks, int64_t sample_batch = 0) {
        size_t o = 0;
        partials = o; o += align_up((size_t)nblocks * kHashMlp * sizeof(float));
        loss_partials = o; o += align_up((size_t)nblocks * sizeof(float));
        grad = o; o += align_up((size_t)np * sizeof(float));
        loss = o; o += align_up(sizeof(float));
        gacc = o; o += align_up((size_t)(np - kHashMlp) * sizeof(unsigned long long));
        gflag = o; o += align_up(sizeof(uint32_t));
        samples = o; o += align_up((size_t)sample_batch * 7 * sizeof(float));
        total = o;
    }
};

nirc_status check_hash_config(const nirc_config *cfg, const nirc_hash_grid *grid, HashGridArgs *args) {
    if (!cfg || !grid) return NIRC_ERR_INVALID_ARG;
    if (cfg->width != 64 || (cfg->precision != NIRC_FP32 && cfg->precision != NIRC_BF16 && cfg->precision != NIRC_FP16) ||
        (cfg->loss != NIRC_LOSS_REL_L2 && cfg->loss != NIRC_LOSS_L2) || cfg->output != NIRC_OUTPUT_RADIANCE)
        return NIRC_ERR_UNSUPPORTED;
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->adam_eps > 0.0f) || !(cfg->loss_eps > 0.0f) ||
        !(cfg->loss_scale > 0.0f))
        return NIRC_ERR_INVALID_ARG;
    if (hash_grid_setup(*grid, args) == 0) return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

int64_t hash_np(const HashGridArgs &g) { return (int64_t)kHashMlp + 2 * (int64_t)g.entries; }

nirc_status check_points_h(const nirc_points &p) {
    if (p.count < 0 || p.count > INT32_MAX) return NIRC_ERR_INVALID_ARG;
    if (p.count > 0 && (!p.px || !p.py || !p.pz || !p.nx || !p.ny || !p.nz || !p.rough)) return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

nirc_status check_queries_h(const nirc_queries &q, const nirc_points &p) {
    if (q.count < 0 || q.count > INT32_MAX) return NIRC_ERR_INVALID_ARG;
    if (q.count > 0 && (!q.wx || !q.wy || !q.wz)) return NIRC_ERR_INVALID_ARG;
    if (q.count > 0 && p.count == 0) return NIRC_ERR_INVALID_ARG;
    if (!q.point && q.count > p.count) return NIRC_ERR_INVALID_ARG;
    return NIRC_OK;
}

Points pts_of(const nirc_points &p) { return Points{p.px, p.py, p.pz, p.nx, p.ny, p.nz, p.rough, p.count}; }
// err: where a point index out of range is reported (sticky flags, or the step's flags)
Queries queries_of(const nirc_queries &q, uint32_t *err) { return Queries{q.wx, q.wy, q.wz, q.point, q.count, err}; }
nirc_status hip_st(hipError_t e) { return e == hipSuccess ? NIRC_OK : NIRC_ERR_HIP; }

}  // namespace

struct nirc_hash_model {
    nirc_config cfg;
    HashGridArgs grid;
    int64_t np;
    float *master, *m, *v;
    uint16_t *packed16;   // the packed layers (FP32 elements for FP32 models)
    int64_t *step;
    uint32_t *flags, *bad;
    char *ws;
    size_t ws_bytes;
    const float *table() const { return master + kHashMlp; }
    float *packed32() const { return (float *)packed16; }
};

namespace {
hipError_t repack(const nirc_hash_model *m, hipStream_t s) {
    return m->cfg.precision == NIRC_FP32 ? launch_hash_pack32(m->packed32(), m->master, s)
                                         : launch_hash_pack16(m->packed16, m->master, m->cfg.precision, s);
}
}  // namespace

extern "C" {

int64_t nirc_hash_entries(const nirc_hash_grid *grid) { return grid ? hash_grid_setup(*grid, nullptr) : 0; }

int64_t nirc_hash_n_params(const nirc_hash_grid *grid) {
    const int64_t e = nirc_hash_entries(grid);
    return e ? (int64_t)kHashMlp + 2 * e : 0;
}

nirc_status nirc_hash_levels(const nirc_hash_grid *grid, int32_t *res, int64_t *offset, int32_t *dense) {
    HashGridArgs g;
    if (!grid || !res || !offset || !dense || hash_grid_setup(*grid, &g) == 0) return NIRC_ERR_INVALID_ARG;
    for (int l = 0; l < kHashLevels; ++l) {
        res[l] = g.lv[l].res;
        offset[l] = g.lv[l].off;
        dense[l] = (int32_t)g.lv[l].dense;
    }
    return NIRC_OK;
}

size_t nirc_hash_state_bytes(const nirc_config *cfg, const nirc_hash_grid *grid) {
    HashGridArgs g;
    if (check_hash_config(cfg, grid, &g) != NIRC_OK) return 0;
    return HashState(hash_np(g), cfg->precision).total;
}

size_t nirc_hash_workspace_bytes(const nirc_config *cfg, const nirc_hash_grid *grid, int64_t max_batch) {
    HashGridArgs g;
    if (check_hash_config(cfg, grid, &g) != NIRC_OK || max_batch < 0) return 0;
    return HashWork(hash_np(g), train_blocks16(max_batch), max_batch).total;
}

nirc_status nirc_hash_create(const nirc_config *cfg, const nirc_hash_grid *grid, void *state, size_t state_bytes,
                             void *workspace, size_t workspace_bytes, const float *init_w, void *stream,
                             nirc_hash_model **out) {
    HashGridArgs g;
    nirc_status st = check_hash_config(cfg, grid, &g);
    if (st != NIRC_OK) return st;
    if (!state || !init_w || !out || ((uintptr_t)state % kAlign) != 0) return NIRC_ERR_INVALID_ARG;
    if (workspace && ((uintptr_t)workspace % kAlign) != 0) return NIRC_ERR_INVALID_ARG;
    const int64_t np = hash_np(g);
    const HashState sl(np, cfg->precision);
    if (state_bytes < sl.total) return NIRC_ERR_WORKSPACE;
    nirc_hash_model *m = new (std::nothrow) nirc_hash_model;
    if (!m) return NIRC_ERR_INVALID_ARG;
    char *base = (char *)state;
    m->cfg = *cfg;
    m->grid = g;
    m->np = np;
    m->master = (float *)(base + sl.master);
    m->m = (float *)(base + sl.m);
    m->v = (float *)(base + sl.v);
    m->packed16 = (uint16_t *)(base + sl.packed16);
    m->step = (int64_t *)(base + sl.step);
    m->flags = (uint32_t *)(base + sl.flags);
    m->bad = (uint32_t *)(base + sl.bad);
    m->ws = (char *)workspace;
    m->ws_bytes = workspace ? workspace_bytes : 0;
    st = nirc_hash_set_weights(m, init_w, stream);
    if (st == NIRC_OK) {
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = launch_fill_u32(m->flags, 1, 0u, s);
        if (e == hipSuccess) e = launch_fill_u32(m->bad, 1, 0u, s);
        st = hip_st(e);
    }
    if (st != NIRC_OK) {
        delete m;
        return st;
    }
    *out = m;
    return NIRC_OK;
}

nirc_status nirc_hash_destroy(nirc_hash_model *model) {
    delete model;
    return NIRC_OK;
}

nirc_status nirc_hash_set_weights(nirc_hash_model *model, const float *w, void *stream) {
    if (!model || !w) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_copy_f32(model->master, w, model->np, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->m, model->np, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->v, model->np, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32((uint32_t *)model->step, 2, 0u, s);
    if (e == hipSuccess) e = repack(model, s);
    return hip_st(e);
}

nirc_status nirc_hash_get_weights(const nirc_hash_model *model, float *w, void *stream) {
    if (!model || !w) return NIRC_ERR_INVALID_ARG;
    return hip_st(launch_copy_f32(w, model->master, model->np, (hipStream_t)stream));
}

// The state is one region from the FP32 parameters on (HashState); a blob is its image.
nirc_status nirc_hash_get_state(const nirc_hash_model *model, void *blob, size_t blob_bytes, void *stream) {
    if (!model || !blob || ((uintptr_t)blob % 4) != 0) return NIRC_ERR_INVALID_ARG;
    const size_t bytes = HashState(model->np, model->cfg.precision).total;
    if (blob_bytes != bytes) return NIRC_ERR_INVALID_ARG;
    return hip_st(launch_copy_f32((float *)blob, model->master, (int64_t)(bytes / 4), (hipStream_t)stream));
}

nirc_status nirc_hash_set_state(nirc_hash_model *model, const void *blob, size_t blob_bytes, void *stream) {
    if (!model || !blob || ((uintptr_t)blob % 4) != 0) return NIRC_ERR_INVALID_ARG;
    const size_t bytes = HashState(model->np, model->cfg.precision).total;
    if (blob_bytes != bytes) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_copy_f32(model->master, (const float *)blob, (int64_t)(bytes / 4), s);
    // the packed layers follow the restored FP32 parameters
    if (e == hipSuccess) e = repack(model, s);
    return hip_st(e);
}

nirc_status nirc_hash_infer(const nirc_hash_model *model, nirc_points points, nirc_queries queries, float *rgb,
                            void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points_h(points);
    if (st == NIRC_OK) st = check_queries_h(queries, points);
    if (st != NIRC_OK) return st;
    if (queries.count == 0) return NIRC_OK;
    if (!rgb) return NIRC_ERR_INVALID_ARG;
    if (model->cfg.precision == NIRC_FP32)
        return hip_st(launch_hash_infer32(pts_of(points), queries_of(queries, model->flags), model->packed32(), model->table(),
                                          model->grid, rgb, (hipStream_t)stream));
    return hip_st(launch_hash_infer(model->cfg.precision, pts_of(points), queries_of(queries, model->flags),
                                    model->packed16, model->table(), model->grid, rgb, (hipStream_t)stream));
}

nirc_status nirc_hash_estimate(const nirc_hash_model *model, nirc_points points, const nirc_lobes *field,
                               int32_t n_cache, uint64_t seed, uint64_t frame, const float *residual_radiance,
                               float *out_tl, float *out_c, float *out_r, void *stream) {
    if (!model || (!field && !residual_radiance)) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points_h(points);
    if (st != NIRC_OK) return st;
    if (n_cache < 1 || n_cache > 4096 || (points.count > 0 && !out_tl)) return NIRC_ERR_INVALID_ARG;
    if (points.count == 0) return NIRC_OK;
    nirc_lobes none;
    memset(&none, 0, sizeof(none));
    if (model->cfg.precision == NIRC_FP32)
        return hip_st(launch_hash_tlmc32(pts_of(points), field ? *field : none, model->packed32(), model->table(),
                                         model->grid, n_cache, seed, frame, residual_radiance, out_tl, out_c, out_r,
                                         (hipStream_t)stream));
    return hip_st(launch_hash_tlmc(model->cfg.precision, pts_of(points), field ? *field : none, model->packed16,
                                   model->table(), model->grid, n_cache, seed, frame, residual_radiance, out_tl, out_c,
                                   out_r, (hipStream_t)stream));
}

// Loss and gradient into grad/loss; the step's `bad` flag is raised on a non-finite value.
static nirc_status hash_grad_into(nirc_hash_model *model, const nirc_points &points, const nirc_queries &queries,
                                  const float *target, float *grad, float *loss, uint32_t *err, hipStream_t s) {
    nirc_status st = check_points_h(points);
    if (st == NIRC_OK) st = check_queries_h(queries, points);
    if (st != NIRC_OK) return st;
    if (queries.count < 1 || !grad || !target) return NIRC_ERR_INVALID_ARG;
    const int nb = train_blocks16(queries.count);
    const HashWork wl(model->np, nb);
    if (!model->ws || model->ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    float *partials = (float *)(model->ws + wl.partials);
    float *lpart = (float *)(model->ws + wl.loss_partials);
    // the batch size is folded into the loss scale (per-sample deltas near unit magnitude in the
    // 16-bit operands; the FP32 kernel takes the same convention); the reductions divide it out again
    const float scale = model->cfg.loss_scale * (float)queries.count;
    const TrainArgs a{target, nullptr, model->cfg.loss_eps, scale, model->cfg.loss, nullptr, 0};
    const int64_t nt = model->np - kHashMlp;
    float *gtab = grad + kHashMlp;
    const GridAcc ga{(unsigned long long *)(model->ws + wl.gacc), (uint32_t *)(model->ws + wl.gflag)};
    hipError_t e = launch_fill_u32((uint32_t *)ga.acc, 2 * nt, 0u, s);
    if (e == hipSuccess) e = launch_fill_u32(ga.nonfinite, 1, 0u, s);
    if (e == hipSuccess)
        e = model->cfg.precision == NIRC_FP32
                ? launch_hash_grad32(pts_of(points), queries_of(queries, err), model->packed32(), model->table(),
                                     model->grid, a, partials, lpart, ga, nb, s)
                : launch_hash_grad(model->cfg.precision, pts_of(points), queries_of(queries, err), model->packed16,
                                   model->table(), model->grid, a, partials, lpart, ga, nb, s);
    if (e == hipSuccess)
        e = launch_reduce_grad_n(kHashMlp, partials, lpart, nb, 1.0f / scale, 1.0f / (3.0f * (float)queries.count),
                                 grad, loss, model->bad, s);
    if (e == hipSuccess) e = launch_grid_acc_finish(ga, gtab, nt, 1.0f / scale, model->bad, s);
    return hip_st(e);
}

static hipError_t hash_adam(nirc_hash_model *model, const float *grad, hipStream_t s) {
    hipError_t e = launch_adam_n(model->np, model->master, model->m, model->v, grad, model->step, model->bad,
                                 model->cfg.lr, model->cfg.beta1, model->cfg.beta2, model->cfg.adam_eps, s);
    if (e == hipSuccess)
        e = model->cfg.precision == NIRC_FP32
                ? launch_hash_pack32(model->packed32(), model->master, s, model->step, model->flags, model->bad)
                : launch_hash_pack16(model->packed16, model->master, model->cfg.precision, s, model->step,
                                     model->flags, model->bad);
    return e;
}

nirc_status nirc_hash_loss_grad(nirc_hash_model *model, nirc_points points, nirc_queries queries,
                                const float *target, float *grad, float *loss, void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    nirc_status st = hash_grad_into(model, points, queries, target, grad, loss, model->flags, s);
    if (st != NIRC_OK) return st;
    // a standalone gradient does not start a step: clear the step's flag again
    return hip_st(launch_fill_u32(model->bad, 1, 0u, s));
}

nirc_status nirc_hash_adam_step(nirc_hash_model *model, const float *grad, void *stream) {
    if (!model || !grad) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = launch_check_finite_n(model->np, grad, model->bad, s);
    if (e == hipSuccess) e = hash_adam(model, grad, s);
    return hip_st(e);
}

nirc_status nirc_hash_train_step(nirc_hash_model *model, nirc_points points, nirc_queries queries,
                                 const float *target, float *loss, void *stream) {
    if (!model) return NIRC_ERR_INVALID_ARG;
    hipStream_t s = (hipStream_t)stream;
    if (!model->ws) return NIRC_ERR_WORKSPACE;
    const HashWork wl(model->np, train_blocks16(queries.count > 0 ? queries.count : 1));
    if (model->ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    float *grad = (float *)(model->ws + wl.grad);
    nirc_status st = hash_grad_into(model, points, queries, target, grad, loss, model->bad, s);
    if (st != NIRC_OK) return st;
    return hip_st(hash_adam(model, grad, s));
}

nirc_status nirc_hash_train_frame(nirc_hash_model *model, nirc_points points, const nirc_lobes *field,
                                  int64_t batch, int32_t steps, uint64_t seed, uint64_t frame, float *loss,
                                  void *stream) {
    if (!model || !field || batch < 1 || batch > INT32_MAX || steps < 0) return NIRC_ERR_INVALID_ARG;
    nirc_status st = check_points_h(points);
    if (st != NIRC_OK || points.count < 1) return NIRC_ERR_INVALID_ARG;
    const HashWork wl(model->np, train_blocks16(batch), batch);
    if (!model->ws || model->ws_bytes < wl.total) return NIRC_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    float *smp = (float *)(model->ws + wl.samples);
    int32_t *pidx = (int32_t *)smp;
    float *wx = smp + batch, *wy = wx + batch, *wz = wy + batch, *tgt = wz + batch;
    for (int32_t k = 0; k < steps; ++k) {
        if (launch_train_batch(pts_of(points), *field, batch, seed, frame, (uint32_t)k, NIRC_OUTPUT_RADIANCE, pidx,
                               wx, wy, wz, tgt, s) != hipSuccess)
            return NIRC_ERR_HIP;
        const nirc_queries q{wx, wy, wz, pidx, batch};
        st = nirc_hash_train_step(model, points, q, tgt, k + 1 == steps ? loss : nullptr, s);
        if (st != NIRC_OK) return st;
    }
    return NIRC_OK;
}

uint32_t nirc_hash_read_flags(const nirc_hash_model *model, void *stream) {
    if (!model) return 0xFFFFFFFFu;
    uint32_t f = 0;
    if (hipMemcpyAsync(&f, model->flags, sizeof(f), hipMemcpyDeviceToHost, (hipStream_t)stream) != hipSuccess)
        return 0xFFFFFFFFu;
    if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) return 0xFFFFFFFFu;
    return f;
}

}  // extern "C"
