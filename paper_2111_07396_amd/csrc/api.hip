// C ABI (include/ssgpu.h): argument validation, launch planning, workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ssgpu.h"
#include "ssgpu_internal.hpp"

namespace ssg {

// Default trial-group shape for a light curve of n points: the smallest
// listed shape that holds it.
int default_shape(int64_t n) {
    static const int order[][3] = {{64, 1, 1},    {128, 1, 2},  {256, 2, 2},   {384, 2, 3},
                                   {512, 4, 2},   {1024, 4, 4}, {2048, 8, 4},  {3072, 16, 3},
                                   {4096, 16, 4}};
    for (const auto &o : order)
        if (n <= o[0])
            for (int s = 0; s < kNumShapes; ++s)
                if (kShapes[s].nw == o[1] && kShapes[s].ppl == o[2]) return s;
    return -1;
}

}  // namespace ssg

using namespace ssg;

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string &msg) {
    g_last_error = msg;
    return code;
}

// A device buffer that only grows.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    hipError_t ensure(size_t want) {
        if (want <= bytes) return hipSuccess;
        if (p) {
            hipError_t e = hipFree(p);
            if (e != hipSuccess) return e;
            p = nullptr;
            bytes = 0;
        }
        size_t sz = std::max<size_t>(want, 256);
        hipError_t e = hipMalloc(&p, sz);
        if (e == hipSuccess) bytes = sz;
        return e;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
};

}  // namespace

struct ss_ctx {
    int device = 0;
    DevBuf tt, w, yc, w32, yc32, chi0, objs, counts, queues, part_p, part_k;
    int max_lds = 65536;
    int n_cu = 1;
    std::vector<std::pair<int32_t, int>> rules;  // (n_max, shape index), sorted by n_max
    int32_t tile_f = 0;
    bool timing = false;
    hipEvent_t ev[2 * kNumShapes] = {};
    int n_timed = 0;
};

#define SS_HIP_TRY(expr, what)                                                               \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess)                                                                \
            return fail(e_ == hipErrorOutOfMemory ? SS_ERR_OOM : SS_ERR_HIP,                 \
                        std::string(what) + ": " + hipGetErrorString(e_));                   \
    } while (0)

namespace {

int check_common(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid, const ss_params *prm) {
    if (!ctx || !cat || !grid || !prm) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (cat->n_obj < 0) return fail(SS_ERR_INVALID_ARG, "n_obj < 0");
    if (cat->n_obj > 0 && (!cat->offsets || !cat->t || !cat->y || !cat->e))
        return fail(SS_ERR_INVALID_ARG, "null catalog pointer");
    if (cat->n_obj > INT32_MAX) return fail(SS_ERR_INVALID_ARG, "n_obj too large");
    if (cat->n_points < 0) return fail(SS_ERR_INVALID_ARG, "n_points < 0");
    if (!(grid->n_freq >= 1) || grid->n_freq > INT32_MAX)
        return fail(SS_ERR_INVALID_ARG, "n_freq must be in [1, 2^31)");
    if (!(std::isfinite(grid->f_min) && std::isfinite(grid->f_max) && grid->f_min > 0.0 &&
          grid->f_max > grid->f_min))
        return fail(SS_ERR_INVALID_ARG, "grid needs 0 < f_min < f_max");
    if (!(prm->span_min > 0.0 && prm->span_min < prm->span_mid &&
          prm->span_mid < prm->span_max && prm->span_max <= 1.0))
        return fail(SS_ERR_INVALID_ARG, "spans need 0 < min < mid < max <= 1");
    if (!(prm->fixed_span >= 0.0 && prm->fixed_span <= 1.0))
        return fail(SS_ERR_INVALID_ARG, "fixed_span must be in [0, 1]");
    if (!std::isfinite(prm->alpha)) return fail(SS_ERR_INVALID_ARG, "alpha must be finite");
    if (prm->precision != SS_FP64 && prm->precision != SS_FP32C)
        return fail(SS_ERR_INVALID_ARG, "precision must be SS_FP64 or SS_FP32C");
    if (prm->flags != 0) return fail(SS_ERR_INVALID_ARG, "flags must be 0");
    return SS_OK;
}

// Chooses the frequency tile: enough (object, tile) items to fill the chip
// several times over, at most 256 trials per item.
int32_t choose_tile(int64_t n_obj, int64_t n_freq) {
    const int64_t target_items = 32768;
    int64_t t = (n_obj * n_freq) / target_items;
    t = std::max<int64_t>(16, std::min<int64_t>(256, t));
    return (int32_t)std::min<int64_t>(t, n_freq);
}

// Runs reset, prep (with device-side planning), one persistent trial launch
// per shape class that can receive objects, and the finalize step.  Nothing
// here waits for the device.
int run(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_grid *grid,
        const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
        int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
        double *best_power) {
    const int64_t n_obj = cat->n_obj;
    if (n_obj == 0) return SS_OK;
    SS_HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    const int64_t total = cat->n_points;
    const int32_t tile = ctx->tile_f > 0 ? (int32_t)std::min<int64_t>(ctx->tile_f, grid->n_freq)
                                         : choose_tile(n_obj, grid->n_freq);
    const int32_t n_tiles = (int32_t)((grid->n_freq + tile - 1) / tile);

    // ---- shape classes: rules, defaults, and which shapes fit in LDS
    const double span_hi = std::max(prm->span_max, prm->fixed_span);
    ShapeRules R{};
    R.max_points = SS_MAX_POINTS;
    R.n_rules = (int32_t)std::min<size_t>(ctx->rules.size(), 16);
    for (int i = 0; i < R.n_rules; ++i) {
        R.rule_n[i] = ctx->rules[(size_t)i].first;
        R.rule_shape[i] = ctx->rules[(size_t)i].second;
    }
    for (int64_t nmax : {64, 128, 256, 384, 512, 1024, 2048, 3072, 4096}) {
        R.def_n[R.n_def] = (int32_t)nmax;
        R.def_shape[R.n_def] = default_shape(nmax);
        R.n_def++;
    }
    std::vector<int32_t> ext(kNumShapes, 2);
    std::vector<bool> used(kNumShapes, false);
    R.runnable = 0u;
    for (int c = 0; c < kNumShapes; ++c) {
        const int np = 64 * kShapes[c].nw * kShapes[c].ppl;
        ext[c] = std::max(2, trial_halfwidth(np, span_hi));
        if (trial_lds_bytes(kShapes[c].nw, kShapes[c].ppl, ext[c]) <= ctx->max_lds)
            R.runnable |= 1u << c;
    }
    R.fallback = default_shape(64);
    for (int i = 0; i < R.n_rules; ++i) used[R.rule_shape[i]] = true;
    for (int i = 0; i < R.n_def; ++i) used[R.def_shape[i]] = true;
    used[R.fallback] = true;

    SS_HIP_TRY(ctx->tt.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->w.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->yc.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->w32.ensure((size_t)total * 4), "workspace");
    SS_HIP_TRY(ctx->yc32.ensure((size_t)total * 4), "workspace");
    SS_HIP_TRY(ctx->chi0.ensure((size_t)n_obj * 8), "workspace");
    SS_HIP_TRY(ctx->objs.ensure((size_t)n_obj * kNumShapes * 4), "workspace");
    SS_HIP_TRY(ctx->counts.ensure((size_t)kNumShapes * 4), "workspace");
    SS_HIP_TRY(ctx->queues.ensure((size_t)kNumShapes * 8), "workspace");
    if (want_best) {
        SS_HIP_TRY(ctx->part_p.ensure((size_t)n_obj * n_tiles * 8), "workspace");
        SS_HIP_TRY(ctx->part_k.ensure((size_t)n_obj * n_tiles * 4), "workspace");
    }
    int32_t *counts = (int32_t *)ctx->counts.p;
    unsigned long long *queues = (unsigned long long *)ctx->queues.p;
    SS_HIP_TRY(launch_reset(counts, queues, kNumShapes, stream), "reset kernel");
    SS_HIP_TRY(launch_prep(cat->offsets, cat->t, cat->y, cat->e, n_obj, total,
                           (double *)ctx->tt.p, (double *)ctx->w.p, (double *)ctx->yc.p,
                           (float *)ctx->w32.p, (float *)ctx->yc32.p, (double *)ctx->chi0.p,
                           obj_status, R, (int32_t *)ctx->objs.p, counts, stream),
               "prep kernel");

    TrialLaunch L{};
    L.cat.offsets = cat->offsets;
    L.cat.tt = (const double *)ctx->tt.p;
    L.cat.w = (const double *)ctx->w.p;
    L.cat.yc = (const double *)ctx->yc.p;
    L.cat.w32 = (const float *)ctx->w32.p;
    L.cat.yc32 = (const float *)ctx->yc32.p;
    L.cat.chi0 = (const double *)ctx->chi0.p;
    L.cat.status = obj_status;
    L.n_tiles = n_tiles;
    L.tile_f = tile;
    L.fmin = grid->f_min;
    L.df = (grid->f_max - grid->f_min) / (double)grid->n_freq;
    L.n_freq = grid->n_freq;
    L.span[0] = prm->span_min;
    L.span[1] = prm->span_mid;
    L.span[2] = prm->span_max;
    L.alpha = prm->alpha;
    L.fixed_span = prm->fixed_span;
    L.method = method;
    L.pgram64 = pgram64;
    L.pgram32 = pgram32;
    L.part_p = want_best ? (double *)ctx->part_p.p : nullptr;
    L.part_k = want_best ? (int32_t *)ctx->part_k.p : nullptr;
    ctx->n_timed = 0;
    for (int c = 0; c < kNumShapes; ++c) {
        if (!used[c] || !((R.runnable >> c) & 1u)) continue;
        TrialLaunch Lc = L;
        Lc.objs = (const int32_t *)ctx->objs.p + (int64_t)c * n_obj;
        Lc.count = counts + c;
        Lc.queue = queues + c;
        Lc.ext = ext[c];
        if (ctx->timing)
            SS_HIP_TRY(hipEventRecord(ctx->ev[2 * ctx->n_timed], stream), "timing event");
        SS_HIP_TRY(launch_trials(shape_id(kShapes[c].nw, kShapes[c].ppl), prm->precision, Lc,
                                 n_obj * (int64_t)n_tiles, ctx->n_cu, stream),
                   "trial kernel");
        if (ctx->timing) {
            SS_HIP_TRY(hipEventRecord(ctx->ev[2 * ctx->n_timed + 1], stream), "timing event");
            ctx->n_timed++;
        }
    }
    if (want_best) {
        SS_HIP_TRY(launch_finalize((const double *)ctx->part_p.p, (const int32_t *)ctx->part_k.p,
                                   n_obj, n_tiles, obj_status, L.fmin, L.df, best_idx,
                                   best_period, best_power, stream),
                   "finalize kernel");
    }
    return SS_OK;
}

}  // namespace

extern "C" {

void ss_params_default(ss_params *p) {
    if (!p) return;
    p->span_min = 0.05;
    p->span_mid = 0.2;
    p->span_max = 0.5;
    p->alpha = 9.0;
    p->fixed_span = 0.0;
    p->precision = SS_FP64;
    p->flags = 0;
}

int ss_ctx_create(int device, ss_ctx **out) {
    if (!out) return fail(SS_ERR_INVALID_ARG, "null out");
    *out = nullptr;
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess) return fail(SS_ERR_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
    if (device < 0 || device >= count) return fail(SS_ERR_INVALID_ARG, "no such device");
    ss_ctx *c = new ss_ctx();
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) ==
            hipSuccess &&
        lds > 0)
        c->max_lds = lds;
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
        ncu > 0)
        c->n_cu = ncu;
    *out = c;
    return SS_OK;
}

void ss_ctx_destroy(ss_ctx *ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    ctx->tt.release();
    ctx->w.release();
    ctx->yc.release();
    ctx->w32.release();
    ctx->yc32.release();
    ctx->chi0.release();
    ctx->objs.release();
    ctx->part_p.release();
    ctx->part_k.release();
    ctx->counts.release();
    ctx->queues.release();
    if (ctx->timing)
        for (auto &e : ctx->ev) (void)hipEventDestroy(e);
    delete ctx;
}

int ss_periodogram(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                   const ss_params *params, void *pgram, int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (cat->n_obj > 0 && (!pgram || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    bool f64 = params->precision == SS_FP64;
    return run(ctx, SS_METHOD_SS, cat, grid, params, f64 ? (double *)pgram : nullptr,
               f64 ? nullptr : (float *)pgram, false, obj_status, (hipStream_t)stream, nullptr,
               nullptr, nullptr);
}

int sssp_periodogram(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                     const ss_params *params, void *pgram, int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (cat->n_obj > 0 && (!pgram || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    bool f64 = params->precision == SS_FP64;
    return run(ctx, SS_METHOD_SSSP, cat, grid, params, f64 ? (double *)pgram : nullptr,
               f64 ? nullptr : (float *)pgram, false, obj_status, (hipStream_t)stream, nullptr,
               nullptr, nullptr);
}

int ss_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat, const ss_grid *grid,
                   const ss_params *params, int64_t *best_idx, double *best_period,
                   double *best_power, int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS or SS_METHOD_SSSP");
    if (cat->n_obj > 0 && (!best_idx || !best_period || !best_power || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    return run(ctx, method, cat, grid, params, nullptr, nullptr, true, obj_status,
               (hipStream_t)stream, best_idx, best_period, best_power);
}

int ss_num_shapes(void) { return kNumShapes; }

int ss_shape_info(int index, int32_t *nw, int32_t *ppl) {
    if (index < 0 || index >= kNumShapes || !nw || !ppl)
        return fail(SS_ERR_INVALID_ARG, "bad shape index");
    *nw = kShapes[index].nw;
    *ppl = kShapes[index].ppl;
    return SS_OK;
}

int ss_ctx_set_shape(ss_ctx *ctx, int32_t n_max, int32_t nw, int32_t ppl) {
    if (!ctx) return fail(SS_ERR_INVALID_ARG, "null context");
    if (nw == 0) {
        ctx->rules.clear();
        return SS_OK;
    }
    int idx = -1;
    for (int s = 0; s < kNumShapes; ++s)
        if (kShapes[s].nw == nw && kShapes[s].ppl == ppl) idx = s;
    if (idx < 0) return fail(SS_ERR_UNSUPPORTED, "shape not built in");
    if (n_max < 1 || n_max > 64 * nw * ppl || n_max > SS_MAX_POINTS)
        return fail(SS_ERR_UNSUPPORTED, "shape too small for n_max");
    for (auto &r : ctx->rules)
        if (r.first == n_max) {
            r.second = idx;
            return SS_OK;
        }
    ctx->rules.emplace_back(n_max, idx);
    std::sort(ctx->rules.begin(), ctx->rules.end());
    return SS_OK;
}

int ss_ctx_set_tile(ss_ctx *ctx, int32_t tile_f) {
    if (!ctx || tile_f < 0) return fail(SS_ERR_INVALID_ARG, "bad tile");
    ctx->tile_f = tile_f;
    return SS_OK;
}

int ss_ctx_set_timing(ss_ctx *ctx, int enable) {
    if (!ctx) return fail(SS_ERR_INVALID_ARG, "null context");
    SS_HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    if (enable && !ctx->timing) {
        for (auto &e : ctx->ev) SS_HIP_TRY(hipEventCreate(&e), "hipEventCreate");
    }
    ctx->timing = enable != 0;
    ctx->n_timed = 0;
    return SS_OK;
}

int ss_ctx_trial_kernel_ms(ss_ctx *ctx, double *ms, int32_t *n_launches) {
    if (!ctx || !ms || !n_launches) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (!ctx->timing) return fail(SS_ERR_INVALID_ARG, "timing is off");
    double total = 0.0;
    for (int i = 0; i < ctx->n_timed; ++i) {
        SS_HIP_TRY(hipEventSynchronize(ctx->ev[2 * i + 1]), "hipEventSynchronize");
        float t = 0.0f;
        SS_HIP_TRY(hipEventElapsedTime(&t, ctx->ev[2 * i], ctx->ev[2 * i + 1]),
                   "hipEventElapsedTime");
        total += t;
    }
    *ms = total;
    *n_launches = ctx->n_timed;
    return SS_OK;
}

const char *ss_last_error(void) { return g_last_error.c_str(); }

int ss_version(void) { return 100; }

}  // extern "C"
