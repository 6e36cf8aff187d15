// C ABI (include/ssgpu.h): argument validation, launch planning, workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ssgpu.h"
#include "ssgpu_internal.hpp"

namespace ssg {

// Default trial-group shape for a light curve of n points: per method and
// precision, the fastest shape measured on MI355X for each length range
// (synthetic catalogs; each kernel with its own register budget, see
// trial_impl.hpp): single-wavefront groups while one wavefront holds the curve at
// up to 3 points per thread, then two wavefronts for FP64 SS and one wavefront
// at 4 points for the single-pass methods and compensated-FP32 SS (whose
// pair sums need twice the registers), wider groups above.
struct ShapeRow {
    int32_t n_max, nw, ppl;
};
constexpr ShapeRow kDefSS64[] = {{64, 1, 1},   {128, 1, 2},  {192, 1, 3},  {256, 2, 2},
                                 {384, 4, 2},  {512, 4, 2},  {1024, 8, 2}, {2048, 8, 4},
                                 {3072, 16, 3}, {4096, 16, 4}};
constexpr ShapeRow kDefSS32[] = {{64, 1, 1},   {128, 1, 2},  {192, 1, 3},  {256, 1, 4},
                                 {384, 2, 3},  {512, 4, 2},  {1024, 4, 4}, {2048, 8, 4},
                                 {3072, 16, 3}, {4096, 16, 4}};
constexpr ShapeRow kDefSP[] = {{64, 1, 1},   {128, 1, 2},  {192, 1, 3},  {256, 1, 4},
                               {384, 2, 3},  {512, 4, 2},  {1024, 4, 4}, {2048, 8, 4},
                               {3072, 16, 3}, {4096, 16, 4}};
constexpr int kNumDefRows = (int)(sizeof(kDefSP) / sizeof(kDefSP[0]));
static_assert(kNumDefRows == (int)(sizeof(kDefSS64) / sizeof(kDefSS64[0])) &&
                  kNumDefRows == (int)(sizeof(kDefSS32) / sizeof(kDefSS32[0])),
              "tables");

int shape_index(int nw, int ppl) {
    for (int s = 0; s < kNumShapes; ++s)
        if (kShapes[s].nw == nw && kShapes[s].ppl == ppl) return s;
    return -1;
}

const ShapeRow *default_rows(int method, int precision) {
    if (method != 0) return kDefSP;
    return precision == SS_FP64 ? kDefSS64 : kDefSS32;
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
    DevBuf tt, w, yc, w32, yc32, chi0, sw, objs, counts, queues, part_p, part_k;
    DevBuf emb, act, logits, dlog, loss_o, dE, partial, ranges, bin_k, scores;
    double bin_grid[3] = {0.0, 0.0, 0.0};  // grid whose bin table is in bin_k
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

// Everything a launch over a catalog needs after prep.
struct Plan {
    ShapeRules R{};
    std::vector<int32_t> ext;
    std::vector<bool> used;
};

// Reset plus prep (with device-side planning of the shape classes).  Nothing
// here waits for the device.
int prepare(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_params *prm,
            int32_t *obj_status, hipStream_t stream, Plan &P) {
    const int64_t n_obj = cat->n_obj;
    const int64_t total = cat->n_points;
    SS_HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    const double span_hi = std::max(prm->span_max, prm->fixed_span);
    ShapeRules &R = P.R;
    R.max_points = SS_MAX_POINTS;
    R.n_rules = (int32_t)std::min<size_t>(ctx->rules.size(), 16);
    for (int i = 0; i < R.n_rules; ++i) {
        R.rule_n[i] = ctx->rules[(size_t)i].first;
        R.rule_shape[i] = ctx->rules[(size_t)i].second;
    }
    const ShapeRow *rows = default_rows(method, prm->precision);
    for (int i = 0; i < kNumDefRows; ++i) {
        R.def_n[R.n_def] = rows[i].n_max;
        R.def_shape[R.n_def] = shape_index(rows[i].nw, rows[i].ppl);
        R.n_def++;
    }
    P.ext.assign(kNumShapes, 2);
    P.used.assign(kNumShapes, false);
    R.runnable = 0u;
    for (int c = 0; c < kNumShapes; ++c) {
        const int np = 64 * kShapes[c].nw * kShapes[c].ppl;
        P.ext[c] = std::max(2, trial_halfwidth(np, span_hi));
        if (trial_lds_bytes(kShapes[c].nw, kShapes[c].ppl, P.ext[c], method) <= ctx->max_lds)
            R.runnable |= 1u << c;
    }
    R.fallback = shape_index(1, 1);
    for (int i = 0; i < R.n_rules; ++i) P.used[R.rule_shape[i]] = true;
    for (int i = 0; i < R.n_def; ++i) P.used[R.def_shape[i]] = true;
    P.used[R.fallback] = true;

    SS_HIP_TRY(ctx->tt.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->w.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->yc.ensure((size_t)total * 8), "workspace");
    SS_HIP_TRY(ctx->w32.ensure((size_t)total * 4), "workspace");
    SS_HIP_TRY(ctx->yc32.ensure((size_t)total * 4), "workspace");
    SS_HIP_TRY(ctx->chi0.ensure((size_t)n_obj * 8), "workspace");
    SS_HIP_TRY(ctx->sw.ensure((size_t)n_obj * 8), "workspace");
    SS_HIP_TRY(ctx->objs.ensure((size_t)n_obj * kNumShapes * 4), "workspace");
    SS_HIP_TRY(ctx->counts.ensure((size_t)kNumShapes * 4), "workspace");
    SS_HIP_TRY(ctx->queues.ensure((size_t)kNumShapes * 8), "workspace");
    int32_t *counts = (int32_t *)ctx->counts.p;
    unsigned long long *queues = (unsigned long long *)ctx->queues.p;
    SS_HIP_TRY(launch_reset(counts, queues, kNumShapes, stream), "reset kernel");
    SS_HIP_TRY(launch_prep(cat->offsets, cat->t, cat->y, cat->e, n_obj, total,
                           (double *)ctx->tt.p, (double *)ctx->w.p, (double *)ctx->yc.p,
                           (float *)ctx->w32.p, (float *)ctx->yc32.p, (double *)ctx->chi0.p,
                           (double *)ctx->sw.p, obj_status, R, (int32_t *)ctx->objs.p, counts,
                           stream),
               "prep kernel");
    return SS_OK;
}

// One persistent trial launch per shape class that can receive objects,
// over n_tiles items per object (full-grid tiles, or refine ranges), then
// the finalize step when the best period is wanted.
int trials(ss_ctx *ctx, const Plan &P, int method, const ss_catalog *cat, const ss_grid *grid,
           const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
           int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
           double *best_power, int32_t tile, int32_t n_tiles, const int64_t *ranges,
           void *pdm = nullptr, int32_t pdm_bins = 0) {
    const int64_t n_obj = cat->n_obj;
    if (want_best) {
        SS_HIP_TRY(ctx->part_p.ensure((size_t)n_obj * n_tiles * 8), "workspace");
        SS_HIP_TRY(ctx->part_k.ensure((size_t)n_obj * n_tiles * 4), "workspace");
    }
    int32_t *counts = (int32_t *)ctx->counts.p;
    unsigned long long *queues = (unsigned long long *)ctx->queues.p;
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
    L.ranges = ranges;
    L.pdm64 = (pdm && prm->precision == SS_FP64) ? (double *)pdm : nullptr;
    L.pdm32 = (pdm && prm->precision != SS_FP64) ? (float *)pdm : nullptr;
    L.pdm_bins = pdm_bins;
    ctx->n_timed = 0;
    for (int c = 0; c < kNumShapes; ++c) {
        if (!P.used[c] || !((P.R.runnable >> c) & 1u)) continue;
        TrialLaunch Lc = L;
        Lc.objs = (const int32_t *)ctx->objs.p + (int64_t)c * n_obj;
        Lc.count = counts + c;
        Lc.queue = queues + c;
        Lc.ext = P.ext[c];
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

// Full-grid search: prep, trials over frequency tiles, finalize.
int run(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_grid *grid,
        const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
        int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
        double *best_power, void *pdm = nullptr, int32_t pdm_bins = 0) {
    const int64_t n_obj = cat->n_obj;
    if (n_obj == 0) return SS_OK;
    const int32_t tile = ctx->tile_f > 0 ? (int32_t)std::min<int64_t>(ctx->tile_f, grid->n_freq)
                                         : choose_tile(n_obj, grid->n_freq);
    const int32_t n_tiles = (int32_t)((grid->n_freq + tile - 1) / tile);
    Plan P;
    int rc = prepare(ctx, method, cat, prm, obj_status, stream, P);
    if (rc != SS_OK) return rc;
    return trials(ctx, P, method, cat, grid, prm, pgram64, pgram32, want_best, obj_status, stream,
                  best_idx, best_period, best_power, tile, n_tiles, nullptr, pdm, pdm_bins);
}

// First fine-grid index of each of the 1024 log-spaced bins over
// [f_min, f_max), and the end of the grid: bin b holds the k with
// E_b <= f_k < E_{b+1}, E_b = f_min (f_max / f_min)^(b / 1024).
void bin_table(const ss_grid *grid, int64_t *first_k) {
    const double df = (grid->f_max - grid->f_min) / (double)grid->n_freq;
    const double ratio = grid->f_max / grid->f_min;
    first_k[0] = 0;
    for (int b = 1; b < kEncBins; ++b) {
        const double edge = grid->f_min * std::pow(ratio, (double)b / (double)kEncBins);
        int64_t k = (int64_t)std::ceil((edge - grid->f_min) / df);
        k = std::max<int64_t>(0, std::min<int64_t>(k, grid->n_freq));
        while (k < grid->n_freq && grid_freq(grid->f_min, df, k) < edge) ++k;
        while (k > 0 && grid_freq(grid->f_min, df, k - 1) >= edge) --k;
        first_k[b] = k;
    }
    first_k[kEncBins] = grid->n_freq;
}

// Feature frequencies: 32 log-spaced over [f_min, f_max], ends included.
void feature_freqs(const ss_grid *grid, double *g) {
    const double a = std::log(grid->f_min), b = std::log(grid->f_max);
    for (int m = 0; m < kEncNFreq; ++m)
        g[m] = (m == kEncNFreq - 1) ? grid->f_max
                                    : std::exp(a + (b - a) * (double)m / (double)(kEncNFreq - 1));
}

int upload_bin_table(ss_ctx *ctx, const ss_grid *grid) {
    if (ctx->bin_k.p && ctx->bin_grid[0] == grid->f_min && ctx->bin_grid[1] == grid->f_max &&
        ctx->bin_grid[2] == (double)grid->n_freq)
        return SS_OK;
    std::vector<int64_t> tab(kEncBins + 1);
    bin_table(grid, tab.data());
    SS_HIP_TRY(ctx->bin_k.ensure(tab.size() * 8), "workspace");
    SS_HIP_TRY(hipMemcpy(ctx->bin_k.p, tab.data(), tab.size() * 8, hipMemcpyHostToDevice),
               "bin table upload");
    ctx->bin_grid[0] = grid->f_min;
    ctx->bin_grid[1] = grid->f_max;
    ctx->bin_grid[2] = (double)grid->n_freq;
    return SS_OK;
}

EncArgs enc_args(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid, const float *params,
                 const int32_t *status) {
    EncArgs A{};
    A.n_obj = (int)cat->n_obj;
    A.offsets = cat->offsets;
    A.tt = (const double *)ctx->tt.p;
    A.yc = (const double *)ctx->yc.p;
    A.e = cat->e;
    A.chi0 = (const double *)ctx->chi0.p;
    A.sw = (const double *)ctx->sw.p;
    A.status = status;
    A.params = params;
    feature_freqs(grid, A.g);
    return A;
}

// Prep, encoder forward and head: logits [n_obj][1024] in ctx->logits
// (or in `logits_out` when given).  act is filled when want_act.
int encode(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_grid *grid,
           const ss_params *prm, const float *params, int32_t *obj_status, hipStream_t stream,
           float *emb_out, float *logits_out, bool want_act, Plan &P, EncArgs &A) {
    const int64_t n_obj = cat->n_obj;
    int rc = prepare(ctx, method, cat, prm, obj_status, stream, P);
    if (rc != SS_OK) return rc;
    SS_HIP_TRY(ctx->emb.ensure((size_t)n_obj * kEncH2 * 4), "workspace");
    SS_HIP_TRY(ctx->act.ensure((size_t)n_obj * kEncH2 * 4), "workspace");
    SS_HIP_TRY(ctx->logits.ensure((size_t)n_obj * kEncBins * 4), "workspace");
    A = enc_args(ctx, cat, grid, params, obj_status);
    A.emb = emb_out ? emb_out : (float *)ctx->emb.p;
    A.act = want_act ? (float *)ctx->act.p : nullptr;
    SS_HIP_TRY(launch_enc_fwd(A, ctx->n_cu, stream), "encoder kernel");
    SS_HIP_TRY(launch_head_fwd(A.emb, params, (int)n_obj,
                               logits_out ? logits_out : (float *)ctx->logits.p, stream),
               "head kernel");
    return SS_OK;
}

// Refine: the planner turns logits into per-object fine-grid ranges and the
// trial kernel searches only those.
int refine(ss_ctx *ctx, const Plan &P, int method, const ss_catalog *cat, const ss_grid *grid,
           const ss_params *prm, const float *logits, const float *scores, float gamma,
           int top_k, int margin, int full_below, int32_t *obj_status, hipStream_t stream,
           int64_t *best_idx, double *best_period, double *best_power) {
    const int64_t n_obj = cat->n_obj;
    int rc = upload_bin_table(ctx, grid);
    if (rc != SS_OK) return rc;
    // Bound on the ranges per object: every run of selected bins holds a top
    // bin, so there are at most top_k runs, each cut into pieces of `chunk`.
    std::vector<int64_t> tab(kEncBins + 1);
    bin_table(grid, tab.data());
    std::vector<int64_t> widths(kEncBins);
    for (int b = 0; b < kEncBins; ++b) widths[b] = tab[b + 1] - tab[b];
    std::sort(widths.begin(), widths.end(), std::greater<int64_t>());
    const int n_sel = std::min(kEncBins, top_k * (2 * margin + 1));
    int64_t max_len = 0;
    for (int i = 0; i < n_sel; ++i) max_len += widths[i];
    max_len = std::min<int64_t>(max_len, grid->n_freq);
    const int32_t chunk = 128;
    int64_t n_rng64 = top_k + (max_len + chunk - 1) / chunk;
    if (full_below > 0) n_rng64 = std::max<int64_t>(n_rng64, (grid->n_freq + chunk - 1) / chunk);
    if (n_rng64 > INT32_MAX / 2) return fail(SS_ERR_INVALID_ARG, "refine set too large");
    const int32_t n_rng = (int32_t)n_rng64;
    SS_HIP_TRY(ctx->ranges.ensure((size_t)n_obj * n_rng * 16), "workspace");
    SS_HIP_TRY(launch_plan(logits, scores, gamma, obj_status, cat->offsets, full_below,
                           (const int64_t *)ctx->bin_k.p, (int)n_obj, top_k, margin, chunk,
                           n_rng, (int64_t *)ctx->ranges.p, stream),
               "refine planner");
    return trials(ctx, P, method, cat, grid, prm, nullptr, nullptr, true, obj_status, stream,
                  best_idx, best_period, best_power, chunk, n_rng,
                  (const int64_t *)ctx->ranges.p);
}

// Cheap exact-grid scores of every log bin into ctx->scores (after prep).
int bin_scores(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid, int32_t *obj_status,
               hipStream_t stream, float *out) {
    int rc = upload_bin_table(ctx, grid);
    if (rc != SS_OK) return rc;
    ScoreArgs A{};
    A.n_obj = (int)cat->n_obj;
    A.offsets = cat->offsets;
    A.tt = (const double *)ctx->tt.p;
    A.w = (const double *)ctx->w.p;
    A.yc = (const double *)ctx->yc.p;
    A.chi0 = (const double *)ctx->chi0.p;
    A.status = obj_status;
    A.bin_k = (const int64_t *)ctx->bin_k.p;
    A.fmin = grid->f_min;
    A.df = (grid->f_max - grid->f_min) / (double)grid->n_freq;
    A.n_freq = grid->n_freq;
    A.scores = out;
    SS_HIP_TRY(launch_bin_scores(A, ctx->n_cu, stream), "bin score kernel");
    return SS_OK;
}

int check_learned(const ss_catalog *cat, int top_k, int margin, int full_below = 0) {
    if (full_below < 0) return fail(SS_ERR_INVALID_ARG, "full_below must be >= 0");
    if (cat->n_obj > 0 && cat->n_obj > INT32_MAX / kEncBins)
        return fail(SS_ERR_INVALID_ARG, "n_obj too large for the encoder");
    if (top_k < 1 || top_k > kEncBins) return fail(SS_ERR_INVALID_ARG, "top_k must be in [1, 1024]");
    if (margin < 0 || margin > 64) return fail(SS_ERR_INVALID_ARG, "margin must be in [0, 64]");
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
    ctx->sw.release();
    for (DevBuf *b : {&ctx->emb, &ctx->act, &ctx->logits, &ctx->dlog, &ctx->loss_o, &ctx->dE,
                      &ctx->partial, &ctx->ranges, &ctx->bin_k, &ctx->scores})
        b->release();
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

int ss_method_periodogram(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                          const ss_grid *grid, const ss_params *params, void *pgram,
                          int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!pgram || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    bool f64 = params->precision == SS_FP64;
    return run(ctx, method, cat, grid, params, f64 ? (double *)pgram : nullptr,
               f64 ? nullptr : (float *)pgram, false, obj_status, (hipStream_t)stream, nullptr,
               nullptr, nullptr);
}

int ss_pdm_periodogram(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                       const ss_grid *grid, const ss_params *params, int32_t n_bins,
                       void *pgram, void *pgram_pdm, int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (n_bins < 0 || n_bins > 256) return fail(SS_ERR_INVALID_ARG, "n_bins must be in [0, 256]");
    if (n_bins == 1) return fail(SS_ERR_INVALID_ARG, "n_bins = 1 explains nothing");
    if (cat->n_obj > 0 && (!pgram || !pgram_pdm || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    bool f64 = params->precision == SS_FP64;
    return run(ctx, method, cat, grid, params, f64 ? (double *)pgram : nullptr,
               f64 ? nullptr : (float *)pgram, false, obj_status, (hipStream_t)stream, nullptr,
               nullptr, nullptr, pgram_pdm, n_bins);
}

int ss_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat, const ss_grid *grid,
                   const ss_params *params, int64_t *best_idx, double *best_period,
                   double *best_power, int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
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

int ss_enc_forward(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                   const float *enc_params, float *emb, float *logits, int32_t *obj_status,
                   void *stream) {
    ss_params prm;
    ss_params_default(&prm);
    int rc = check_common(ctx, cat, grid, &prm);
    if (rc != SS_OK) return rc;
    rc = check_learned(cat, 1, 0);
    if (rc != SS_OK) return rc;
    if (cat->n_obj > 0 && (!enc_params || !emb || !logits || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null argument");
    if (cat->n_obj == 0) return SS_OK;
    Plan P;
    EncArgs A;
    return encode(ctx, SS_METHOD_SS, cat, grid, &prm, enc_params, obj_status,
                  (hipStream_t)stream, emb, logits, false, P, A);
}

int ss_enc_train_grad(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                      const float *enc_params, const int32_t *labels, float *grad, float *loss,
                      int32_t *obj_status, void *stream) {
    ss_params prm;
    ss_params_default(&prm);
    int rc = check_common(ctx, cat, grid, &prm);
    if (rc != SS_OK) return rc;
    rc = check_learned(cat, 1, 0);
    if (rc != SS_OK) return rc;
    if (cat->n_obj < 1) return fail(SS_ERR_INVALID_ARG, "training needs n_obj >= 1");
    if (!enc_params || !labels || !grad || !loss || !obj_status)
        return fail(SS_ERR_INVALID_ARG, "null argument");
    const hipStream_t s = (hipStream_t)stream;
    const int64_t n_obj = cat->n_obj;
    Plan P;
    EncArgs A;
    rc = encode(ctx, SS_METHOD_SS, cat, grid, &prm, enc_params, obj_status, s, nullptr, nullptr,
                true, P, A);
    if (rc != SS_OK) return rc;
    const int n_waves = enc_bwd_waves((int)n_obj, ctx->n_cu);
    SS_HIP_TRY(ctx->dlog.ensure((size_t)n_obj * kEncBins * 4), "workspace");
    SS_HIP_TRY(ctx->loss_o.ensure((size_t)n_obj * 4), "workspace");
    SS_HIP_TRY(ctx->dE.ensure((size_t)n_obj * kEncH2 * 4), "workspace");
    SS_HIP_TRY(ctx->partial.ensure((size_t)n_waves * enc_mlp_grad_floats() * 4), "workspace");
    A.partial = (float *)ctx->partial.p;
    SS_HIP_TRY(launch_train_tail(A, (const float *)ctx->logits.p, labels, (float *)ctx->dlog.p,
                                 (float *)ctx->loss_o.p, (float *)ctx->dE.p, grad, loss, n_waves,
                                 s),
               "training kernels");
    return SS_OK;
}

int ss_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream) {
    if (n < 0 || (n > 0 && (!params || !grad || !m || !v)))
        return fail(SS_ERR_INVALID_ARG, "null argument");
    if (step < 1) return fail(SS_ERR_INVALID_ARG, "step counts from 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps >= 0.0f &&
          std::isfinite(lr)))
        return fail(SS_ERR_INVALID_ARG, "bad Adam hyper-parameters");
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    SS_HIP_TRY(launch_adam(params, grad, m, v, n, lr, beta1, beta2, eps, c1, c2,
                           (hipStream_t)stream),
               "adam kernel");
    return SS_OK;
}

int ss_refine_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                          const ss_grid *grid, const ss_params *params, const float *logits,
                          int32_t top_k, int32_t margin, int32_t full_below, int64_t *best_idx,
                          double *best_period, double *best_power, int32_t *obj_status,
                          void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    rc = check_learned(cat, top_k, margin, full_below);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!logits || !best_idx || !best_period || !best_power || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null argument");
    if (cat->n_obj == 0) return SS_OK;
    const hipStream_t s = (hipStream_t)stream;
    Plan P;
    rc = prepare(ctx, method, cat, params, obj_status, s, P);
    if (rc != SS_OK) return rc;
    return refine(ctx, P, method, cat, grid, params, logits, nullptr, 0.0f, top_k, margin,
                  full_below, obj_status, s, best_idx, best_period, best_power);
}

int ss_learned_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, const float *enc_params,
                           float gamma, int32_t top_k, int32_t margin, int32_t full_below,
                           int64_t *best_idx, double *best_period, double *best_power,
                           int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    rc = check_learned(cat, top_k, margin, full_below);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (!std::isfinite(gamma) || gamma < 0.0f)
        return fail(SS_ERR_INVALID_ARG, "gamma must be finite and >= 0");
    if (!enc_params && gamma == 0.0f)
        return fail(SS_ERR_INVALID_ARG, "no proposal: enc_params is null and gamma is 0");
    if (cat->n_obj > 0 && (!best_idx || !best_period || !best_power || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null argument");
    if (cat->n_obj == 0) return SS_OK;
    const hipStream_t s = (hipStream_t)stream;
    const int64_t n_obj = cat->n_obj;
    Plan P;
    const float *logits = nullptr;
    if (enc_params) {
        EncArgs A;
        rc = encode(ctx, method, cat, grid, params, enc_params, obj_status, s, nullptr, nullptr,
                    false, P, A);
        if (rc != SS_OK) return rc;
        logits = (const float *)ctx->logits.p;
    } else {
        rc = prepare(ctx, method, cat, params, obj_status, s, P);
        if (rc != SS_OK) return rc;
    }
    const float *scores = nullptr;
    if (gamma > 0.0f) {
        SS_HIP_TRY(ctx->scores.ensure((size_t)n_obj * kEncBins * 4), "workspace");
        rc = bin_scores(ctx, cat, grid, obj_status, s, (float *)ctx->scores.p);
        if (rc != SS_OK) return rc;
        scores = (const float *)ctx->scores.p;
    }
    return refine(ctx, P, method, cat, grid, params, logits, scores, gamma, top_k, margin,
                  full_below, obj_status, s, best_idx, best_period, best_power);
}

int ss_bin_scores(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid, float *scores,
                  int32_t *obj_status, void *stream) {
    ss_params prm;
    ss_params_default(&prm);
    int rc = check_common(ctx, cat, grid, &prm);
    if (rc != SS_OK) return rc;
    rc = check_learned(cat, 1, 0);
    if (rc != SS_OK) return rc;
    if (cat->n_obj > 0 && (!scores || !obj_status)) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (cat->n_obj == 0) return SS_OK;
    const hipStream_t s = (hipStream_t)stream;
    Plan P;
    rc = prepare(ctx, SS_METHOD_SS, cat, &prm, obj_status, s, P);
    if (rc != SS_OK) return rc;
    return bin_scores(ctx, cat, grid, obj_status, s, scores);
}

int ss_bin_table(const ss_grid *grid, int64_t *first_k) {
    if (!grid || !first_k) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (!(grid->n_freq >= 1) || grid->n_freq > INT32_MAX)
        return fail(SS_ERR_INVALID_ARG, "n_freq must be in [1, 2^31)");
    if (!(std::isfinite(grid->f_min) && std::isfinite(grid->f_max) && grid->f_min > 0.0 &&
          grid->f_max > grid->f_min))
        return fail(SS_ERR_INVALID_ARG, "grid needs 0 < f_min < f_max");
    bin_table(grid, first_k);
    return SS_OK;
}

int ss_enc_num_params(void) { return kEncParams; }

const char *ss_last_error(void) { return g_last_error.c_str(); }

int ss_version(void) { return 140; }

}  // extern "C"
