// C ABI (include/ssgpu.h): argument validation, launch planning, workspace.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <functional>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
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
// pair sums need twice the registers), wider groups above (FP64 SS up to 384
// points on two wavefronts at 3 points per thread: 9.2e7 trials/s at
// N = 300 against 5.7e7 on four wavefronts at 2).
struct ShapeRow {
    int32_t n_max, nw, ppl;
};
constexpr ShapeRow kDefSS64[] = {{64, 1, 1},   {128, 1, 2},  {192, 1, 3},  {256, 2, 2},
                                 {384, 2, 3},  {512, 4, 2},  {1024, 8, 2}, {2048, 8, 4},
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

// Device pointers of one call's workspace: the context's own buffers, or a
// fixed region (the allocation-free entry point).
struct Work {
    double *tt = nullptr, *w = nullptr, *yc = nullptr;
    float *w32 = nullptr, *yc32 = nullptr;
    double *chi0 = nullptr, *sw = nullptr;
    int32_t *objs = nullptr, *counts = nullptr;
    unsigned long long *queues = nullptr;
    double *part_p = nullptr;
    int32_t *part_k = nullptr;
};

struct ss_ctx {
    int device = 0;
    void *noalloc = nullptr;       // this device's copy of the fixed region
    Work cur;                      // workspace of the call in progress
    const Work *fixed = nullptr;   // when set: use it, never allocate
    DevBuf tt, w, yc, w32, yc32, chi0, sw, objs, counts, queues, part_p, part_k;
    DevBuf emb, act, logits, dlog, loss_o, dE, partial, ranges, bin_k, scores;
    DevBuf sh_offsets, sh_tt;  // shared time sampling: CSR offsets o*n, t - min t
    double bin_grid[3] = {0.0, 0.0, 0.0};  // grid whose bin table is in bin_k
    int max_lds = 65536;
    int n_cu = 1;
    std::vector<std::pair<int32_t, int>> rules;  // (n_max, shape index), sorted by n_max
    int32_t tile_f = 0;
    bool timing = false;
    hipEvent_t ev[2 * kNumShapes] = {};
    int n_timed = 0;
    // class launches of one call run concurrently: forked from the caller's
    // stream onto these (default-priority) streams and joined back to it
    bool forked = false;
    // fork the class launches of a call (off by default: measured on MI355X,
    // the serial launches are faster -- N=200 SS 1.64e8 vs 1.44e8 trials/s,
    // uneven catalog 1.35e8 vs 1.23e8 -- as the launches of empty classes,
    // which wait for resources behind the busy ones, hold up the join)
    bool concurrent = false;
    hipStream_t side[kNumShapes] = {};
    hipEvent_t fork_ev = nullptr, join_ev[kNumShapes] = {};
    int64_t chunk_bytes = 0;  // batched periodogram: the current output chunk
    DevBuf chunk;
    DevBuf dbg;                      // debug mode: device counters of the invariant checks
    unsigned long long dbg_host[4] = {0, 0, 0, 0};  // their staging copy on the host
    int64_t check_counts[3] = {0, 0, 0};  // their values after the last checked call
};

// A learned frequency proposal bound to one search grid: the encoder's FP32
// master parameters, Adam moments and step count, all on the device of the
// context that made it.
struct ss_model {
    int device = 0;
    ss_grid grid{};
    int32_t step = 0;
    float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
    DevBuf params, m, v, grad;
};

// ---- the fixed region of the allocation-free entry point
// Device memory that ss_best_period_noalloc uses in place of the context's
// growing workspace.  Every device the library runs on holds its own copy
// until the process ends; host code never uses the array's name as an
// address, only the per-device address resolved by hipGetSymbolAddress.
constexpr size_t kNoAllocBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];
static_assert(kNoAllocBytes == (size_t)SS_NOALLOC_BYTES, "header and library agree");

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

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
    if ((prm->flags & ~(SS_FLAG_CHECK_INVARIANTS | SS_FLAG_CHECK_SELFTEST)) != 0)
        return fail(SS_ERR_INVALID_ARG, "unknown flag bits");
    if ((prm->flags & SS_FLAG_CHECK_SELFTEST) && !(prm->flags & SS_FLAG_CHECK_INVARIANTS))
        return fail(SS_ERR_INVALID_ARG, "SS_FLAG_CHECK_SELFTEST needs SS_FLAG_CHECK_INVARIANTS");
    return SS_OK;
}

// Entry points other than the full-grid searches take no debug flags.
int no_flags(const ss_params *prm) {
    if (prm && prm->flags != 0)
        return fail(SS_ERR_INVALID_ARG, "debug flags are taken by the full-grid calls only");
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

int check_grid(const ss_grid *grid) {
    if (!grid) return fail(SS_ERR_INVALID_ARG, "null grid");
    if (!(grid->n_freq >= 1) || grid->n_freq > INT32_MAX)
        return fail(SS_ERR_INVALID_ARG, "n_freq must be in [1, 2^31)");
    if (!(std::isfinite(grid->f_min) && std::isfinite(grid->f_max) && grid->f_min > 0.0 &&
          grid->f_max > grid->f_min))
        return fail(SS_ERR_INVALID_ARG, "grid needs 0 < f_min < f_max");
    return SS_OK;
}

// Objects per work item under shared time sampling (at most kMaxSharedBatch).
constexpr int32_t kSharedBatch = 8;
static_assert(kSharedBatch <= kMaxSharedBatch, "shared batch");

// Everything a launch over a catalog needs after prep.
struct Plan {
    ShapeRules R{};
    std::vector<int32_t> ext;
    std::vector<bool> used;
};

// Reset plus prep (with device-side planning of the shape classes).  Nothing
// here waits for the device.
int prepare(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_params *prm,
            int32_t *obj_status, hipStream_t stream, Plan &P, bool shared_t = false) {
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

    if (ctx->fixed) {
        ctx->cur = *ctx->fixed;
    } else {
        SS_HIP_TRY(ctx->tt.ensure((size_t)total * 8), "workspace");
        SS_HIP_TRY(ctx->w.ensure((size_t)total * 8), "workspace");
        SS_HIP_TRY(ctx->yc.ensure((size_t)total * 8), "workspace");
        SS_HIP_TRY(ctx->w32.ensure((size_t)total * 4), "workspace");
        SS_HIP_TRY(ctx->yc32.ensure((size_t)total * 4), "workspace");
        SS_HIP_TRY(ctx->chi0.ensure((size_t)n_obj * 8), "workspace");
        SS_HIP_TRY(ctx->sw.ensure((size_t)n_obj * 8), "workspace");
        SS_HIP_TRY(ctx->objs.ensure((size_t)n_obj * kNumShapes * 4), "workspace");
        SS_HIP_TRY(ctx->counts.ensure((size_t)kNumShapes * 4), "workspace");
        SS_HIP_TRY(ctx->queues.ensure((size_t)kNumShapes * kQueuesPerClass * 8), "workspace");
        Work &W = ctx->cur;
        W.tt = (double *)ctx->tt.p;
        W.w = (double *)ctx->w.p;
        W.yc = (double *)ctx->yc.p;
        W.w32 = (float *)ctx->w32.p;
        W.yc32 = (float *)ctx->yc32.p;
        W.chi0 = (double *)ctx->chi0.p;
        W.sw = (double *)ctx->sw.p;
        W.objs = (int32_t *)ctx->objs.p;
        W.counts = (int32_t *)ctx->counts.p;
        W.queues = (unsigned long long *)ctx->queues.p;
    }
    int32_t *counts = ctx->cur.counts;
    unsigned long long *queues = ctx->cur.queues;
    SS_HIP_TRY(launch_reset(counts, queues, kNumShapes, stream), "reset kernel");
    SS_HIP_TRY(launch_prep(cat->offsets, cat->t, cat->y, cat->e, n_obj, total,
                           ctx->cur.tt, ctx->cur.w, ctx->cur.yc, ctx->cur.w32, ctx->cur.yc32,
                           ctx->cur.chi0, ctx->cur.sw, obj_status, R, ctx->cur.objs, counts,
                           stream, shared_t),
               "prep kernel");
    return SS_OK;
}

int ensure_side_streams(ss_ctx *ctx) {
    if (ctx->forked) return SS_OK;
    for (int i = 0; i < kNumShapes; ++i) {
        SS_HIP_TRY(hipStreamCreateWithFlags(&ctx->side[i], hipStreamNonBlocking), "stream");
        SS_HIP_TRY(hipEventCreateWithFlags(&ctx->join_ev[i], hipEventDisableTiming), "event");
    }
    SS_HIP_TRY(hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming), "event");
    ctx->forked = true;
    return SS_OK;
}

// The launch description common to the classes of one call (no outputs).
TrialLaunch base_launch(const ss_ctx *ctx, int method, const ss_catalog *cat,
                        const ss_grid *grid, const ss_params *prm, int32_t *obj_status,
                        int32_t tile, int32_t n_tiles) {
    TrialLaunch L{};
    L.cat.offsets = cat->offsets;
    L.cat.tt = ctx->cur.tt;
    L.cat.w = ctx->cur.w;
    L.cat.yc = ctx->cur.yc;
    L.cat.w32 = ctx->cur.w32;
    L.cat.yc32 = ctx->cur.yc32;
    L.cat.chi0 = ctx->cur.chi0;
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
    return L;
}

// Class c's part of a launch: its object list, count, queues and extension.
TrialLaunch class_launch(const TrialLaunch &L, const ss_ctx *ctx, const Plan &P, int c,
                         int64_t n_obj) {
    TrialLaunch Lc = L;
    Lc.objs = ctx->cur.objs + (int64_t)c * n_obj;
    Lc.count = ctx->cur.counts + c;
    Lc.queue = ctx->cur.queues + (size_t)c * kQueuesPerClass;
    Lc.ext = P.ext[c];
    return Lc;
}

// Debug mode (SS_FLAG_CHECK_INVARIANTS): after the trials, the invariant
// check kernels over the same items and classes; waits for the device and
// fails with SS_ERR_INVARIANT when a sorted key or a window weight is wrong.
int run_checks(ss_ctx *ctx, const Plan &P, int method, const ss_catalog *cat,
               const ss_grid *grid, const ss_params *prm, int32_t *obj_status,
               hipStream_t stream, int32_t tile, int32_t n_tiles) {
    const int64_t n_obj = cat->n_obj;
    SS_HIP_TRY(ctx->dbg.ensure(4 * sizeof(unsigned long long)), "workspace");
    unsigned long long *d = (unsigned long long *)ctx->dbg.p;
    unsigned long long *h = ctx->dbg_host;  // lives as long as the context
    for (int i = 0; i < 4; ++i) h[i] = 0;
    SS_HIP_TRY(hipMemcpyAsync(d, h, 4 * sizeof(*h), hipMemcpyHostToDevice, stream),
               "debug counters");
    const TrialLaunch L = base_launch(ctx, method, cat, grid, prm, obj_status, tile, n_tiles);
    const int selftest = (prm->flags & SS_FLAG_CHECK_SELFTEST) ? 1 : 0;
    for (int c = 0; c < kNumShapes; ++c) {
        if (!P.used[c] || !((P.R.runnable >> c) & 1u)) continue;
        const TrialLaunch Lc = class_launch(L, ctx, P, c, n_obj);
        SS_HIP_TRY(launch_checks(shape_id(kShapes[c].nw, kShapes[c].ppl), Lc,
                                 n_obj * (int64_t)n_tiles, ctx->n_cu, d, selftest, stream),
                   "check kernel");
    }
    SS_HIP_TRY(hipMemcpyAsync(h, d, 4 * sizeof(*h), hipMemcpyDeviceToHost, stream),
               "debug counters");
    SS_HIP_TRY(hipStreamSynchronize(stream), "debug counters");
    for (int i = 0; i < 3; ++i) ctx->check_counts[i] = (int64_t)h[i];
    if (h[1] != 0 || h[2] != 0)
        return fail(SS_ERR_INVARIANT, "invariant check: " + std::to_string(h[1]) +
                                          " sorted keys out of order, " + std::to_string(h[2]) +
                                          " windows with W <= 0, in " + std::to_string(h[0]) +
                                          " trials");
    return SS_OK;
}

// One persistent trial launch per shape class that can receive objects,
// over n_tiles items per object (full-grid tiles, or refine ranges), then
// the finalize step when the best period is wanted.
int trials(ss_ctx *ctx, const Plan &P, int method, const ss_catalog *cat, const ss_grid *grid,
           const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
           int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
           double *best_power, int32_t tile, int32_t n_tiles, const int64_t *ranges,
           void *pdm = nullptr, int32_t pdm_bins = 0, int shared_class = -1,
           int32_t shared_batch = 0, int32_t shared_n = 0, const double *shared_tt = nullptr) {
    const int64_t n_obj = cat->n_obj;
    if (want_best && !ctx->fixed) {
        SS_HIP_TRY(ctx->part_p.ensure((size_t)n_obj * n_tiles * 8), "workspace");
        SS_HIP_TRY(ctx->part_k.ensure((size_t)n_obj * n_tiles * 4), "workspace");
        ctx->cur.part_p = (double *)ctx->part_p.p;
        ctx->cur.part_k = (int32_t *)ctx->part_k.p;
    }
    TrialLaunch L = base_launch(ctx, method, cat, grid, prm, obj_status, tile, n_tiles);
    L.pgram64 = pgram64;
    L.pgram32 = pgram32;
    L.part_p = want_best ? ctx->cur.part_p : nullptr;
    L.part_k = want_best ? ctx->cur.part_k : nullptr;
    L.ranges = ranges;
    L.pdm64 = (pdm && prm->precision == SS_FP64) ? (double *)pdm : nullptr;
    L.pdm32 = (pdm && prm->precision != SS_FP64) ? (float *)pdm : nullptr;
    L.pdm_bins = pdm_bins;
    ctx->n_timed = 0;
    int n_launch = 0;

    for (int c = 0; c < kNumShapes; ++c)
        if (P.used[c] && ((P.R.runnable >> c) & 1u)) ++n_launch;
    // several classes: fork them onto the side streams so that one class's
    // tail overlaps the others' work (timing then covers fork to join)
    const bool fork = n_launch > 1 && !ctx->fixed && ctx->concurrent;
    if (fork) {
        int rc = ensure_side_streams(ctx);
        if (rc != SS_OK) return rc;
        if (ctx->timing) SS_HIP_TRY(hipEventRecord(ctx->ev[0], stream), "timing event");
        SS_HIP_TRY(hipEventRecord(ctx->fork_ev, stream), "fork event");
    }
    int launched = 0;
    for (int c = 0; c < kNumShapes; ++c) {
        if (!P.used[c] || !((P.R.runnable >> c) & 1u)) continue;
        TrialLaunch Lc = class_launch(L, ctx, P, c, n_obj);
        if (c == shared_class) {
            Lc.shared_batch = shared_batch;
            Lc.shared_n = shared_n;
            Lc.shared_tt = shared_tt;
        }
        if (fork) {
            hipStream_t sc = ctx->side[launched];
            SS_HIP_TRY(hipStreamWaitEvent(sc, ctx->fork_ev, 0), "fork");
            SS_HIP_TRY(launch_trials(shape_id(kShapes[c].nw, kShapes[c].ppl), prm->precision,
                                     Lc, n_obj * (int64_t)n_tiles, ctx->n_cu, sc),
                       "trial kernel");
            SS_HIP_TRY(hipEventRecord(ctx->join_ev[launched], sc), "join event");
        } else {
            if (ctx->timing)
                SS_HIP_TRY(hipEventRecord(ctx->ev[2 * ctx->n_timed], stream), "timing event");
            SS_HIP_TRY(launch_trials(shape_id(kShapes[c].nw, kShapes[c].ppl), prm->precision,
                                     Lc, n_obj * (int64_t)n_tiles, ctx->n_cu, stream),
                       "trial kernel");
            if (ctx->timing) {
                SS_HIP_TRY(hipEventRecord(ctx->ev[2 * ctx->n_timed + 1], stream),
                           "timing event");
                ctx->n_timed++;
            }
        }
        ++launched;
    }
    if (fork) {
        for (int i = 0; i < launched; ++i)
            SS_HIP_TRY(hipStreamWaitEvent(stream, ctx->join_ev[i], 0), "join");
        if (ctx->timing) {
            SS_HIP_TRY(hipEventRecord(ctx->ev[1], stream), "timing event");
            ctx->n_timed = 1;
        }
    }
    if (want_best) {
        SS_HIP_TRY(launch_finalize(ctx->cur.part_p, ctx->cur.part_k,
                                   n_obj, n_tiles, obj_status, L.fmin, L.df, best_idx,
                                   best_period, best_power, stream),
                   "finalize kernel");
    }
    return SS_OK;
}

int32_t tile_for(const ss_ctx *ctx, int64_t n_obj, int64_t n_freq) {
    return ctx->tile_f > 0 ? (int32_t)std::min<int64_t>(ctx->tile_f, n_freq)
                           : choose_tile(n_obj, n_freq);
}

// Full-grid search: prep, trials over frequency tiles, finalize.
int run(ss_ctx *ctx, int method, const ss_catalog *cat, const ss_grid *grid,
        const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
        int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
        double *best_power, void *pdm = nullptr, int32_t pdm_bins = 0) {
    const int64_t n_obj = cat->n_obj;
    if (n_obj == 0) return SS_OK;
    const int32_t tile = tile_for(ctx, n_obj, grid->n_freq);
    const int32_t n_tiles = (int32_t)((grid->n_freq + tile - 1) / tile);
    Plan P;
    int rc = prepare(ctx, method, cat, prm, obj_status, stream, P);
    if (rc != SS_OK) return rc;
    rc = trials(ctx, P, method, cat, grid, prm, pgram64, pgram32, want_best, obj_status, stream,
                best_idx, best_period, best_power, tile, n_tiles, nullptr, pdm, pdm_bins);
    if (rc != SS_OK || !(prm->flags & SS_FLAG_CHECK_INVARIANTS)) return rc;
    return run_checks(ctx, P, method, cat, grid, prm, obj_status, stream, tile, n_tiles);
}

// Objects that share one time sampling: a CSR view (offsets o*n, built on
// the device), prep reading the one t array, and one class launch whose
// work items are batches of objects x frequency tiles (fold and sort once
// per trial frequency and batch).  Objects the shape tables cannot run
// (too long, or a shape that does not fit the LDS) take the ordinary path
// of their class, which reports them.
int run_shared(ss_ctx *ctx, int method, const ss_shared_catalog *sc, const ss_grid *grid,
               const ss_params *prm, double *pgram64, float *pgram32, bool want_best,
               int32_t *obj_status, hipStream_t stream, int64_t *best_idx, double *best_period,
               double *best_power) {
    const int64_t n_obj = sc->n_obj, n = sc->n_points;
    if (n_obj == 0) return SS_OK;
    SS_HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
    SS_HIP_TRY(ctx->sh_offsets.ensure((size_t)(n_obj + 1) * 8), "workspace");
    SS_HIP_TRY(ctx->sh_tt.ensure((size_t)std::max<int64_t>(n, 1) * 8), "workspace");
    SS_HIP_TRY(launch_shared_layout(sc->t, n, n_obj, (int64_t *)ctx->sh_offsets.p,
                                    (double *)ctx->sh_tt.p, stream),
               "shared layout kernel");
    ss_catalog cat{n_obj, n_obj * n, (const int64_t *)ctx->sh_offsets.p, sc->t, sc->y, sc->e};
    Plan P;
    int rc = prepare(ctx, method, &cat, prm, obj_status, stream, P, true);
    if (rc != SS_OK) return rc;
    // the class every object of length n is filed in (rules first, then the
    // defaults), as the prep kernel decides it
    int cls = -1;
    for (int i = 0; i < P.R.n_rules && cls < 0; ++i)
        if (n <= P.R.rule_n[i]) cls = P.R.rule_shape[i];
    for (int i = 0; i < P.R.n_def && cls < 0; ++i)
        if (n <= P.R.def_n[i]) cls = P.R.def_shape[i];
    const bool runs = cls >= 0 && n <= P.R.max_points && ((P.R.runnable >> cls) & 1u);
    const int32_t batch = runs ? (int32_t)std::min<int64_t>(kSharedBatch, n_obj) : 0;
    const int64_t units = runs ? (n_obj + batch - 1) / batch : n_obj;
    const int32_t tile = ctx->tile_f > 0 ? (int32_t)std::min<int64_t>(ctx->tile_f, grid->n_freq)
                                         : choose_tile(units, grid->n_freq);
    const int32_t n_tiles = (int32_t)((grid->n_freq + tile - 1) / tile);
    return trials(ctx, P, method, &cat, grid, prm, pgram64, pgram32, want_best, obj_status,
                  stream, best_idx, best_period, best_power, tile, n_tiles, nullptr, nullptr, 0,
                  runs ? cls : -1, batch, (int32_t)n, (const double *)ctx->sh_tt.p);
}

int check_shared(ss_ctx *ctx, const ss_shared_catalog *sc, const ss_grid *grid,
                 const ss_params *prm) {
    if (!sc) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (sc->n_obj < 0 || sc->n_points < 0)
        return fail(SS_ERR_INVALID_ARG, "n_obj and n_points must be >= 0");
    if (sc->n_obj > 0 && sc->n_points > INT64_MAX / sc->n_obj)
        return fail(SS_ERR_INVALID_ARG, "catalog too large");
    // offsets are built on the device; any non-null pointer passes the null check
    ss_catalog cat{sc->n_obj, sc->n_obj * sc->n_points, (const int64_t *)sc->t, sc->t, sc->y,
                   sc->e};
    int rc = check_common(ctx, &cat, grid, prm);
    if (rc != SS_OK) return rc;
    rc = no_flags(prm);
    if (rc != SS_OK) return rc;
    if (sc->n_obj > 0 && sc->n_points > 0 && (!sc->t || !sc->y || !sc->e))
        return fail(SS_ERR_INVALID_ARG, "null catalog pointer");
    return SS_OK;
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
    A.tt = ctx->cur.tt;
    A.yc = ctx->cur.yc;
    A.e = cat->e;
    A.chi0 = ctx->cur.chi0;
    A.sw = ctx->cur.sw;
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
    A.tt = ctx->cur.tt;
    A.w = ctx->cur.w;
    A.yc = ctx->cur.yc;
    A.chi0 = ctx->cur.chi0;
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
    // the fixed region's address on this device, resolved once per device
    // with that device current
    if (device < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[device]) {
            int prev = 0;
            hipError_t ge = hipGetDevice(&prev);
            if (ge == hipSuccess) ge = hipSetDevice(device);
            void *ptr = nullptr;
            if (ge == hipSuccess) ge = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            (void)hipSetDevice(prev);
            if (ge != hipSuccess || !ptr) {
                delete c;
                return fail(SS_ERR_HIP, std::string("hipGetSymbolAddress: ") +
                                            hipGetErrorString(ge));
            }
            g_scratch_ptr[device] = ptr;
        }
        c->noalloc = g_scratch_ptr[device];
    }
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
                      &ctx->partial, &ctx->ranges, &ctx->bin_k, &ctx->scores,
                      &ctx->sh_offsets, &ctx->sh_tt})
        b->release();
    ctx->objs.release();
    ctx->part_p.release();
    ctx->part_k.release();
    ctx->counts.release();
    ctx->queues.release();
    if (ctx->timing)
        for (auto &e : ctx->ev) (void)hipEventDestroy(e);
    if (ctx->forked) {
        for (int i = 0; i < kNumShapes; ++i) {
            (void)hipStreamDestroy(ctx->side[i]);
            (void)hipEventDestroy(ctx->join_ev[i]);
        }
        (void)hipEventDestroy(ctx->fork_ev);
    }
    ctx->chunk.release();
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

int ss_shared_periodogram(ss_ctx *ctx, int32_t method, const ss_shared_catalog *cat,
                          const ss_grid *grid, const ss_params *params, void *pgram,
                          int32_t *obj_status, void *stream) {
    int rc = check_shared(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!pgram || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    bool f64 = params->precision == SS_FP64;
    return run_shared(ctx, method, cat, grid, params, f64 ? (double *)pgram : nullptr,
                      f64 ? nullptr : (float *)pgram, false, obj_status, (hipStream_t)stream,
                      nullptr, nullptr, nullptr);
}

int ss_shared_best_period(ss_ctx *ctx, int32_t method, const ss_shared_catalog *cat,
                          const ss_grid *grid, const ss_params *params, int64_t *best_idx,
                          double *best_period, double *best_power, int32_t *obj_status,
                          void *stream) {
    int rc = check_shared(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!best_idx || !best_period || !best_power || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    return run_shared(ctx, method, cat, grid, params, nullptr, nullptr, true, obj_status,
                      (hipStream_t)stream, best_idx, best_period, best_power);
}

int ss_plan_batches(ss_ctx *ctx, int64_t n_obj, int64_t n_points, const ss_grid *grid,
                    int32_t precision, int32_t want_pgram, double beta, int64_t mem_bytes,
                    int64_t *objs_per_batch, int64_t *n_batches) {
    if (!ctx || !objs_per_batch || !n_batches) return fail(SS_ERR_INVALID_ARG, "null argument");
    int rc = check_grid(grid);
    if (rc != SS_OK) return rc;
    if (n_obj < 0 || n_points < 0) return fail(SS_ERR_INVALID_ARG, "negative size");
    if (precision != SS_FP64 && precision != SS_FP32C)
        return fail(SS_ERR_INVALID_ARG, "precision must be SS_FP64 or SS_FP32C");
    if (!(beta > 0.0 && beta <= 1.0)) return fail(SS_ERR_INVALID_ARG, "beta must be in (0, 1]");
    if (mem_bytes < 0) return fail(SS_ERR_INVALID_ARG, "mem_bytes must be >= 0");
    double s = (double)mem_bytes;
    if (mem_bytes == 0) {
        SS_HIP_TRY(hipSetDevice(ctx->device), "hipSetDevice");
        size_t free_b = 0, total_b = 0;
        SS_HIP_TRY(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
        s = (double)free_b;
    }
    // footprint r = fixed + n_obj * per_obj: the per-point prep workspace
    // (tt, w, yc in FP64, w, yc in FP32) is needed once; per object the
    // output row, the per-tile partials of the best-period reduction and the
    // per-object arrays
    const double fixed = 32.0 * (double)n_points;
    const double row = want_pgram ? (double)grid->n_freq * (precision == SS_FP64 ? 8.0 : 4.0)
                                  : 0.0;
    const int64_t tiles = (grid->n_freq + 15) / 16;  // the smallest automatic tile
    const double per_obj = row + 12.0 * (double)tiles + 16.0 + 4.0 * kNumShapes + 4.0;
    const double room = beta * s - fixed;
    if (room < per_obj)
        return fail(SS_ERR_OOM, "not even one object fits beta times the device memory");
    const int64_t per = (int64_t)std::min<double>(std::floor(room / per_obj),
                                                  (double)std::max<int64_t>(n_obj, 1));
    *objs_per_batch = per;
    *n_batches = n_obj == 0 ? 0 : (n_obj + per - 1) / per;
    return SS_OK;
}

int ss_periodogram_batched(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, void *chunk,
                           int64_t chunk_objs, ss_pgram_sink sink, void *user,
                           int32_t *obj_status, void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!chunk || !sink || !obj_status || chunk_objs < 1))
        return fail(SS_ERR_INVALID_ARG, "null chunk, sink or status, or chunk_objs < 1");
    const hipStream_t st = (hipStream_t)stream;
    const bool f64 = params->precision == SS_FP64;
    for (int64_t lo = 0; lo < cat->n_obj; lo += chunk_objs) {
        const int64_t hi = std::min(cat->n_obj, lo + chunk_objs);
        // offsets are absolute indices into t, y, e: a batch is a window of them
        ss_catalog sub{hi - lo, cat->n_points, cat->offsets + lo, cat->t, cat->y, cat->e};
        rc = run(ctx, method, &sub, grid, params, f64 ? (double *)chunk : nullptr,
                 f64 ? nullptr : (float *)chunk, false, obj_status + lo, st, nullptr, nullptr,
                 nullptr);
        if (rc != SS_OK) return rc;
        SS_HIP_TRY(hipStreamSynchronize(st), "hipStreamSynchronize");
        sink(user, lo, hi, chunk, obj_status + lo);
    }
    return SS_OK;
}

int ss_best_period_noalloc(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, int64_t *best_idx,
                           double *best_period, double *best_power, int32_t *obj_status,
                           void *stream) {
    int rc = check_common(ctx, cat, grid, params);
    if (rc != SS_OK) return rc;
    rc = no_flags(params);
    if (rc != SS_OK) return rc;
    if (method != SS_METHOD_SS && method != SS_METHOD_SSSP && method != SS_METHOD_SSSP_GV)
        return fail(SS_ERR_INVALID_ARG, "method must be SS_METHOD_SS, _SSSP or _SSSP_GV");
    if (cat->n_obj > 0 && (!best_idx || !best_period || !best_power || !obj_status))
        return fail(SS_ERR_INVALID_ARG, "null output pointer");
    if (!ctx->noalloc) return fail(SS_ERR_UNSUPPORTED, "no fixed region on this device");
    const int64_t n_obj = cat->n_obj, total = cat->n_points;
    if (n_obj == 0) return SS_OK;
    const int32_t tile = tile_for(ctx, n_obj, grid->n_freq);
    const int64_t n_tiles = (grid->n_freq + tile - 1) / tile;
    // carve the region as the context's workspace would be laid out
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) {
        const uint64_t at = off;
        off += (bytes + 255) / 256 * 256;
        return (unsigned char *)ctx->noalloc + at;
    };
    Work W;
    W.tt = (double *)take((uint64_t)total * 8);
    W.w = (double *)take((uint64_t)total * 8);
    W.yc = (double *)take((uint64_t)total * 8);
    W.w32 = (float *)take((uint64_t)total * 4);
    W.yc32 = (float *)take((uint64_t)total * 4);
    W.chi0 = (double *)take((uint64_t)n_obj * 8);
    W.sw = (double *)take((uint64_t)n_obj * 8);
    W.objs = (int32_t *)take((uint64_t)n_obj * kNumShapes * 4);
    W.counts = (int32_t *)take((uint64_t)kNumShapes * 4);
    W.queues = (unsigned long long *)take((uint64_t)kNumShapes * kQueuesPerClass * 8);
    W.part_p = (double *)take((uint64_t)n_obj * n_tiles * 8);
    W.part_k = (int32_t *)take((uint64_t)n_obj * n_tiles * 4);
    if (off > kNoAllocBytes)
        return fail(SS_ERR_UNSUPPORTED,
                    "catalog needs " + std::to_string(off) + " bytes of working memory; the "
                    "allocation-free entry point has " + std::to_string(kNoAllocBytes));
    ctx->fixed = &W;
    rc = run(ctx, method, cat, grid, params, nullptr, nullptr, true, obj_status,
             (hipStream_t)stream, best_idx, best_period, best_power);
    ctx->fixed = nullptr;
    return rc;
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

int ss_ctx_set_concurrency(ss_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(SS_ERR_INVALID_ARG, "null context");
    ctx->concurrent = enable != 0;
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
    rc = no_flags(params);
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
    rc = no_flags(params);
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

}  // extern "C"

// ---- model object: parameters, Adam state, save / load

namespace {

constexpr char kModelMagic[8] = {'S', 'S', 'G', 'P', 'U', 'M', 'D', 'L'};
constexpr uint32_t kModelFormat = 1;

// Fixed little-endian header that precedes the JSON metadata and the arrays.
struct ModelHeader {
    char magic[8];
    uint32_t format;
    uint32_t json_bytes;  // JSON text follows the header
    uint64_t n_params;
    int32_t step;
    float beta1, beta2, eps;
    double f_min, f_max;
    int64_t n_freq;
    uint64_t array_offset;  // byte offset of params[n], then m[n], v[n] (float32)
};

bool same_grid(const ss_grid &a, const ss_grid *b) {
    return a.f_min == b->f_min && a.f_max == b->f_max && a.n_freq == b->n_freq;
}

std::string model_json(const ss_model *m) {
    char buf[64];
    std::ostringstream js;
    auto num = [&](double v) {
        std::snprintf(buf, sizeof buf, "%.17g", v);
        return std::string(buf);
    };
    double g[kEncNFreq];
    feature_freqs(&m->grid, g);
    js << "{\"format\": \"ssgpu-model\", \"format_version\": " << kModelFormat
       << ", \"library_version\": " << ss_version() << ", \"n_params\": " << kEncParams
       << ", \"layout\": [[\"W1\", 80, 64], [\"W2\", 64, 128], [\"b2\", 128], "
          "[\"W3\", 128, 1024], [\"b3\", 1024]]"
       << ", \"grid\": {\"f_min\": " << num(m->grid.f_min) << ", \"f_max\": "
       << num(m->grid.f_max) << ", \"n_freq\": " << m->grid.n_freq << "}"
       << ", \"bins\": " << kEncBins
       << ", \"bin_edges\": \"E_b = f_min (f_max / f_min)^(b / 1024)\""
       << ", \"feature_freqs\": [";
    for (int i = 0; i < kEncNFreq; ++i) js << (i ? ", " : "") << num(g[i]);
    js << "], \"step\": " << m->step << ", \"adam\": {\"beta1\": " << num(m->beta1)
       << ", \"beta2\": " << num(m->beta2) << ", \"eps\": " << num(m->eps) << "}"
       << ", \"arrays\": [\"params\", \"adam_m\", \"adam_v\"], \"dtype\": \"float32\"}";
    return js.str();
}

int model_alloc(ss_model *m) {
    const size_t bytes = (size_t)kEncParams * 4;
    SS_HIP_TRY(hipSetDevice(m->device), "hipSetDevice");
    SS_HIP_TRY(m->params.ensure(bytes), "model allocation");
    SS_HIP_TRY(m->m.ensure(bytes), "model allocation");
    SS_HIP_TRY(m->v.ensure(bytes), "model allocation");
    SS_HIP_TRY(m->grad.ensure(bytes), "model allocation");
    return SS_OK;
}

void model_free(ss_model *m) {
    (void)hipSetDevice(m->device);
    m->params.release();
    m->m.release();
    m->v.release();
    m->grad.release();
}

}  // namespace

extern "C" {

int ss_model_create(ss_ctx *ctx, const ss_grid *grid, const float *init_params,
                    ss_model **out) {
    if (!ctx || !out || !init_params) return fail(SS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc != SS_OK) return rc;
    ss_model *m = new ss_model();
    m->device = ctx->device;
    m->grid = *grid;
    rc = model_alloc(m);
    const size_t bytes = (size_t)kEncParams * 4;
    if (rc == SS_OK) {
        hipError_t e = hipMemcpy(m->params.p, init_params, bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(m->m.p, 0, bytes);
        if (e == hipSuccess) e = hipMemset(m->v.p, 0, bytes);
        if (e != hipSuccess)
            rc = fail(SS_ERR_HIP, std::string("model upload: ") + hipGetErrorString(e));
    }
    if (rc != SS_OK) {
        model_free(m);
        delete m;
        return rc;
    }
    *out = m;
    return SS_OK;
}

void ss_model_destroy(ss_model *model) {
    if (!model) return;
    model_free(model);
    delete model;
}

int ss_model_info(const ss_model *model, ss_grid *grid, int32_t *step,
                  const float **device_params) {
    if (!model) return fail(SS_ERR_INVALID_ARG, "null model");
    if (grid) *grid = model->grid;
    if (step) *step = model->step;
    if (device_params) *device_params = (const float *)model->params.p;
    return SS_OK;
}

int ss_model_copy_params(const ss_model *model, float *dst, void *stream) {
    if (!model || !dst) return fail(SS_ERR_INVALID_ARG, "null argument");
    SS_HIP_TRY(hipSetDevice(model->device), "hipSetDevice");
    SS_HIP_TRY(hipMemcpyAsync(dst, model->params.p, (size_t)kEncParams * 4,
                              hipMemcpyDeviceToDevice, (hipStream_t)stream),
               "parameter copy");
    return SS_OK;
}

int ss_model_file_write(const char *path, const ss_grid *grid, int32_t step,
                        const float *params, const float *adam_m, const float *adam_v) {
    if (!path || !params || !adam_m || !adam_v) return fail(SS_ERR_INVALID_ARG, "null argument");
    int rc = check_grid(grid);
    if (rc != SS_OK) return rc;
    if (step < 0) return fail(SS_ERR_INVALID_ARG, "step must be >= 0");
    ss_model meta;
    meta.grid = *grid;
    meta.step = step;
    const size_t n = (size_t)kEncParams;
    const std::string js = model_json(&meta);
    ModelHeader h{};
    std::memcpy(h.magic, kModelMagic, 8);
    h.format = kModelFormat;
    h.json_bytes = (uint32_t)js.size();
    h.n_params = n;
    h.step = step;
    h.beta1 = meta.beta1;
    h.beta2 = meta.beta2;
    h.eps = meta.eps;
    h.f_min = grid->f_min;
    h.f_max = grid->f_max;
    h.n_freq = grid->n_freq;
    h.array_offset = (sizeof(ModelHeader) + js.size() + 63) / 64 * 64;
    std::ofstream f(path, std::ios::binary | std::ios::trunc);
    if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot open for writing: ") + path);
    f.write((const char *)&h, sizeof h);
    f.write(js.data(), (std::streamsize)js.size());
    const std::string pad(h.array_offset - sizeof h - js.size(), '\n');
    f.write(pad.data(), (std::streamsize)pad.size());
    for (const float *a : {params, adam_m, adam_v}) f.write((const char *)a, (std::streamsize)(n * 4));
    f.close();
    if (!f) return fail(SS_ERR_INVALID_ARG, std::string("write failed: ") + path);
    return SS_OK;
}

int ss_model_file_read(const char *path, ss_grid *grid, int32_t *step, float *params,
                       float *adam_m, float *adam_v) {
    if (!path || !grid || !step || !params || !adam_m || !adam_v)
        return fail(SS_ERR_INVALID_ARG, "null argument");
    std::ifstream f(path, std::ios::binary);
    if (!f) return fail(SS_ERR_INVALID_ARG, std::string("cannot open: ") + path);
    f.seekg(0, std::ios::end);
    const uint64_t size = (uint64_t)f.tellg();
    f.seekg(0, std::ios::beg);
    ModelHeader h{};
    if (size < sizeof h || !f.read((char *)&h, sizeof h))
        return fail(SS_ERR_INVALID_ARG, "not a model file (too short)");
    if (std::memcmp(h.magic, kModelMagic, 8) != 0)
        return fail(SS_ERR_INVALID_ARG, "not a model file (bad magic)");
    if (h.format != kModelFormat)
        return fail(SS_ERR_UNSUPPORTED, "model file format " + std::to_string(h.format) +
                                            " (this library reads " +
                                            std::to_string(kModelFormat) + ")");
    if (h.n_params != (uint64_t)kEncParams)
        return fail(SS_ERR_INVALID_ARG, "model has " + std::to_string(h.n_params) +
                                            " parameters, the encoder needs " +
                                            std::to_string(kEncParams));
    const uint64_t need = h.array_offset + 3ull * h.n_params * 4;
    if (h.array_offset < sizeof h + (uint64_t)h.json_bytes || size < need)
        return fail(SS_ERR_INVALID_ARG, "model file truncated or inconsistent");
    ss_grid g{h.f_min, h.f_max, h.n_freq};
    if (check_grid(&g) != SS_OK) return fail(SS_ERR_INVALID_ARG, "model file has an invalid grid");
    if (h.step < 0 || !(h.beta1 == 0.9f && h.beta2 == 0.999f && h.eps == 1e-8f))
        return fail(SS_ERR_INVALID_ARG, "model file has invalid optimizer state");
    const size_t n = (size_t)h.n_params;
    f.seekg((std::streamoff)h.array_offset, std::ios::beg);
    for (float *a : {params, adam_m, adam_v})
        if (!f.read((char *)a, (std::streamsize)(n * 4)))
            return fail(SS_ERR_INVALID_ARG, "model file truncated");
    *grid = g;
    *step = h.step;
    return SS_OK;
}

int ss_model_save(const ss_model *model, const char *path) {
    if (!model || !path) return fail(SS_ERR_INVALID_ARG, "null argument");
    const size_t n = (size_t)kEncParams;
    std::vector<float> host(3 * n);
    SS_HIP_TRY(hipSetDevice(model->device), "hipSetDevice");
    SS_HIP_TRY(hipDeviceSynchronize(), "hipDeviceSynchronize");
    SS_HIP_TRY(hipMemcpy(host.data(), model->params.p, n * 4, hipMemcpyDeviceToHost),
               "model download");
    SS_HIP_TRY(hipMemcpy(host.data() + n, model->m.p, n * 4, hipMemcpyDeviceToHost),
               "model download");
    SS_HIP_TRY(hipMemcpy(host.data() + 2 * n, model->v.p, n * 4, hipMemcpyDeviceToHost),
               "model download");
    return ss_model_file_write(path, &model->grid, model->step, host.data(), host.data() + n,
                               host.data() + 2 * n);
}

int ss_model_load(ss_ctx *ctx, const char *path, ss_model **out) {
    if (!ctx || !path || !out) return fail(SS_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    const size_t n = (size_t)kEncParams;
    std::vector<float> host(3 * n);
    ss_grid g{};
    int32_t step = 0;
    int rc = ss_model_file_read(path, &g, &step, host.data(), host.data() + n, host.data() + 2 * n);
    if (rc != SS_OK) return rc;
    ss_model *m = new ss_model();
    m->device = ctx->device;
    m->grid = g;
    m->step = step;
    rc = model_alloc(m);
    if (rc == SS_OK) {
        hipError_t e = hipMemcpy(m->params.p, host.data(), n * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(m->m.p, host.data() + n, n * 4, hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(m->v.p, host.data() + 2 * n, n * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess)
            rc = fail(SS_ERR_HIP, std::string("model upload: ") + hipGetErrorString(e));
    }
    if (rc != SS_OK) {
        model_free(m);
        delete m;
        return rc;
    }
    *out = m;
    return SS_OK;
}

int ss_train_step(ss_ctx *ctx, ss_model *model, const ss_catalog *batch, const int32_t *labels,
                  float lr, float *loss, int32_t *obj_status, void *stream) {
    if (!ctx || !model) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (model->device != ctx->device)
        return fail(SS_ERR_INVALID_ARG, "model and context are on different devices");
    if (!std::isfinite(lr)) return fail(SS_ERR_INVALID_ARG, "lr must be finite");
    if (model->step == INT32_MAX) return fail(SS_ERR_UNSUPPORTED, "step counter exhausted");
    int rc = ss_enc_train_grad(ctx, batch, &model->grid, (const float *)model->params.p, labels,
                               (float *)model->grad.p, loss, obj_status, stream);
    if (rc != SS_OK) return rc;
    rc = ss_adam_step((float *)model->params.p, (const float *)model->grad.p,
                      (float *)model->m.p, (float *)model->v.p, kEncParams, model->step + 1, lr,
                      model->beta1, model->beta2, model->eps, stream);
    if (rc != SS_OK) return rc;
    model->step++;
    return SS_OK;
}

int ss_best_period_learned(ss_ctx *ctx, const ss_model *model, int32_t method,
                           const ss_catalog *cat, const ss_grid *grid, const ss_params *params,
                           float gamma, int32_t top_k, int32_t margin, int32_t full_below,
                           int64_t *best_idx, double *best_period, double *best_power,
                           int32_t *obj_status, void *stream) {
    if (!ctx || !model || !grid) return fail(SS_ERR_INVALID_ARG, "null argument");
    if (model->device != ctx->device)
        return fail(SS_ERR_INVALID_ARG, "model and context are on different devices");
    if (!same_grid(model->grid, grid))
        return fail(SS_ERR_INVALID_ARG, "the model was trained for another search grid");
    return ss_learned_best_period(ctx, method, cat, grid, params,
                                  (const float *)model->params.p, gamma, top_k, margin,
                                  full_below, best_idx, best_period, best_power, obj_status,
                                  stream);
}

const char *ss_last_error(void) { return g_last_error.c_str(); }

int ss_version(void) { return 151; }

int ss_ctx_check_counts(ss_ctx *ctx, int64_t *out) {
    if (!ctx || !out) return fail(SS_ERR_INVALID_ARG, "null argument");
    for (int i = 0; i < 3; ++i) out[i] = ctx->check_counts[i];
    return SS_OK;
}

}  // extern "C"
