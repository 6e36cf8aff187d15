// Internal interfaces between the C-ABI host layer and the gfx950 kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssg {

// Prepared catalog (written by the prep kernel into the context workspace).
struct Prepared {
    const int64_t *offsets;  // caller's CSR offsets
    const double *tt;        // t - min(t) per point
    const double *w;         // e^-2 per point
    const double *yc;        // y - weighted mean, per point
    const float *w32;        // FP32 copies for the compensated-FP32 path
    const float *yc32;
    const double *chi0;      // per object
    const int32_t *status;   // per object
};

// One persistent launch of the trial kernel over one shape class.  Work items
// are (object of the class, frequency tile); workgroups take them from a
// device-side queue until count * n_tiles items are done.
struct TrialLaunch {
    Prepared cat;
    const int32_t *objs;         // object ids of this class (written by prep)
    const int32_t *count;        // number of objects in this class
    unsigned long long *queue;   // kQueuesPerClass counters of items handed out
                                 // (zeroed before prep)
    int32_t n_tiles;
    int32_t tile_f;
    double fmin, df;
    int64_t n_freq;
    double span[3];
    double alpha;
    double fixed_span;
    int32_t method;       // 0 SS, 1 SSSP (GCV per trial), 2 SSSP (GV per point)
    int32_t ext;          // periodic extension of the prefix sums (>= every b used)
    double *pgram64;      // [n_obj * n_freq] or null
    float *pgram32;       // [n_obj * n_freq] or null
    double *part_p;       // [n_obj * n_tiles] or null
    int32_t *part_k;      // [n_obj * n_tiles] or null
    const int64_t *ranges;  // refine: [n_obj][n_tiles] of (k_begin, k_end), or null for
                            // the full grid cut into tiles of tile_f
    double *pdm64;          // phase-dispersion periodogram [n_obj * n_freq] or null
    float *pdm32;
    int32_t pdm_bins;       // phase bins (0: clamp(n / 5, 4, 32))
    // shared time sampling: work items are (batch of shared_batch objects of
    // the class, tile); every object has shared_n points observed at the
    // times whose prepared form is shared_tt.  shared_batch = 0: off.
    int32_t shared_batch;
    int32_t shared_n;
    const double *shared_tt;
};
constexpr int kMaxSharedBatch = 16;

// Work queues per size class: one per XCD of MI355X (workgroups are dispatched
// to the 8 XCDs in turn by workgroup id).  Queue q holds the items of the
// class's objects with slot = q mod 8, so all frequency tiles of an object are
// taken on one XCD and its data is fetched into that XCD's L2 once; a
// workgroup whose own queue is empty takes from the others.
constexpr int kQueuesPerClass = 8;

// Expressions that must round exactly like their plain C statement (no
// fused multiply-add), so that grid frequencies, window half-widths and the
// Listing 1 threshold agree bit for bit with a straightforward evaluation.
__host__ __device__ __forceinline__ double grid_freq(double fmin, double df, int64_t k) {
#pragma clang fp contract(off)
    double kd = (double)k;
    double step = kd * df;
    return fmin + step;
}

// 0.5 span n + 0.5, with the product formed as span (n / 2): halving is exact,
// so this is the same rounded product as (0.5 span) n, and no factor of it
// is invariant across work items (a hoisted 0.5 span was held in registers
// for the whole kernel).
__host__ __device__ __forceinline__ double halfwidth_real(double span, int n) {
#pragma clang fp contract(off)
    return span * (0.5 * (double)n) + 0.5;
}

__host__ __device__ __forceinline__ double listing_vsmlsq(double scale) {
#pragma clang fp contract(off)
    return 1.0e-6 * scale * scale;
}

// Trial-group shapes (NW wavefronts, PPL points per thread): a light curve of
// n points runs on any shape with 64*NW*PPL >= n.
#define SSG_SHAPES(X) \
    X(1, 1) X(1, 2) X(2, 1) X(1, 3) X(1, 4) X(2, 2) X(4, 1) X(2, 3) X(4, 2) X(2, 4) X(4, 4) X(8, 2) \
    X(8, 4) X(16, 3) X(16, 4)
constexpr int shape_id(int nw, int ppl) { return nw * 16 + ppl; }
struct ShapeInfo {
    int nw, ppl;
};
constexpr ShapeInfo kShapes[] = {
#define SSG_SHAPE_INFO(nw, ppl) {nw, ppl},
    SSG_SHAPES(SSG_SHAPE_INFO)
#undef SSG_SHAPE_INFO
};
constexpr int kNumShapes = (int)(sizeof(kShapes) / sizeof(kShapes[0]));

int trial_lds_bytes(int nw, int ppl, int ext, int method);  // dynamic LDS of one trial group
int trial_halfwidth(int n, double span);         // window half-width b(n, span)

// Shape selection on the device: the first rule with n <= n_max, else the
// first default entry with n <= n_max.  Objects longer than max_points or
// whose shape is not runnable (LDS) get status SS_OBJ_TOO_LONG and go to
// class `fallback`.
struct ShapeRules {
    int32_t n_rules, n_def, max_points, fallback;
    int32_t rule_n[16], rule_shape[16];
    int32_t def_n[16], def_shape[16];
    uint32_t runnable;  // bit per shape index
};

// Zeroes the per-class object counts and the kQueuesPerClass queue heads of
// each class (a kernel, so that the sequence stays valid inside a captured
// graph).
hipError_t launch_reset(int32_t *counts, unsigned long long *queues, int n, hipStream_t stream);

// Prep plus planning: status, tt/w/yc, chi0, and the object's entry in its
// shape class (objs[class * n_obj + slot], counts[class]).
hipError_t launch_prep(const int64_t *offsets, const double *t, const double *y, const double *e,
                       int64_t n_obj, int64_t n_points, double *tt, double *w, double *yc, float *w32, float *yc32,
                       double *chi0, double *sw, int32_t *status, const ShapeRules &rules,
                       int32_t *objs, int32_t *counts, hipStream_t stream,
                       bool shared_t = false);

// Shared time sampling: offsets[o] = o*n (o <= n_obj) and shared_tt = t - min t.
hipError_t launch_shared_layout(const double *t, int64_t n, int64_t n_obj, int64_t *offsets,
                                double *shared_tt, hipStream_t stream);

// Debug mode: the invariant checks of the trial kernels' sort and windows over
// one class's items; adds to counts[0..2] (trials, unordered sorted keys,
// windows with W <= 0).
hipError_t launch_checks(int shape_id, const TrialLaunch &L, int64_t max_items, int n_cu,
                         unsigned long long *counts, int selftest, hipStream_t s);

// Persistent launch of one class: grid = co-resident workgroups (at most
// max_items).
hipError_t launch_trials(int shape_id, int precision, const TrialLaunch &L, int64_t max_items,
                         int n_cu, hipStream_t stream);

hipError_t launch_finalize(const double *part_p, const int32_t *part_k, int64_t n_obj,
                           int32_t n_tiles, const int32_t *status, double fmin, double df,
                           int64_t *best_idx, double *best_period, double *best_power,
                           hipStream_t stream);

// ---- learned frequency proposal (set encoder) ----
constexpr int kEncK1 = 80, kEncH1 = 64, kEncH2 = 128, kEncBins = 1024, kEncNFreq = 32;
constexpr int kEncParams =
    kEncK1 * kEncH1 + kEncH1 * kEncH2 + kEncH2 + kEncH2 * kEncBins + kEncBins;

struct EncArgs {
    int n_obj;
    const int64_t *offsets;
    const double *tt, *yc, *e, *chi0, *sw;  // prepped catalog (tt, yc, chi0, sw) and raw e
    const int32_t *status;
    const float *params;     // FP32 master parameters
    double g[kEncNFreq];     // feature frequencies
    float *emb, *act;        // [n_obj][128]; act may be null
    const float *dE;         // backward: dL/d emb [n_obj][128]
    float *partial;          // backward: per-wave W1/W2 gradient slots
};

int enc_fwd_lds_bytes();
int enc_bwd_lds_bytes(int waves);
int enc_mlp_grad_floats();
int enc_bwd_waves(int n_obj, int n_cu);
hipError_t launch_enc_fwd(const EncArgs &A, int n_cu, hipStream_t s);
hipError_t launch_head_fwd(const float *emb, const float *prm, int n_obj, float *logits,
                           hipStream_t s);
// Cross-entropy, head gradients, per-point backward and the gradient
// reduction (grad must hold kEncParams floats; every entry is written).
hipError_t launch_train_tail(const EncArgs &A, const float *logits, const int32_t *labels,
                             float *dlog, float *loss_o, float *dE, float *grad, float *loss,
                             int n_waves, hipStream_t s);
hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_plan(const float *logits, const float *scores, float gamma,
                       const int32_t *status, const int64_t *offsets, int full_below,
                       const int64_t *bin_k, int n_obj, int top_k, int margin, int chunk,
                       int n_rng, int64_t *ranges, hipStream_t s);

// Cheap exact-grid proposal score: for every grid frequency the fraction of
// chi0 explained by a phase-binned (piecewise constant) model with
// B = clamp(n / 5, 4, 32) equal phase bins, max-pooled into the 1024 log
// bins of the grid (scores [n_obj][1024], zero for bins without a grid
// frequency and for objects with a nonzero status).
struct ScoreArgs {
    int n_obj;
    const int64_t *offsets;
    const double *tt;     // prepped
    const double *w, *yc;
    const double *chi0;
    const int32_t *status;
    const int64_t *bin_k;  // 1025 first indices of the log bins
    double fmin, df;
    int64_t n_freq;
    float *scores;
};
constexpr int kScoreMaxBins = 32;
hipError_t launch_bin_scores(const ScoreArgs &A, int n_cu, hipStream_t s);

}  // namespace ssg
