/*
 * ssgpu.h -- C ABI of the MI355X (gfx950) Super Smoother period search.
 *
 * Method: Gowanlock, Butler, Trilling & McNeill, "GPU-Enabled Searches for
 * Periodic Signals of Unknown Shape" (arXiv 2111.07396).  For every
 * (object, trial frequency) pair the library folds the light curve at the
 * trial period, sorts it by phase, runs Friedman's variable-span Super
 * Smoother (Listing 1, Sec. 2.2) or the single-pass generalized-validation
 * variant (Sec. 3), scores the fit and reduces the scores to a periodogram
 * and a best period (Alg. 1).
 *
 * Conventions shared by every entry point
 *  - Every data pointer is a DEVICE pointer on the context's device, owned by
 *    the caller.  The library never frees or retains caller memory.
 *  - Calls are asynchronous on the HIP stream passed as `stream`
 *    (hipStream_t, NULL = the default stream).  Outputs are valid once that
 *    stream has been synchronized.  A call never synchronizes or reads device
 *    data on the host: planning (shape classes, work queues) runs on the
 *    device, so a call may be captured into a HIP graph and replayed, once a
 *    first call with the same sizes has grown the context's workspace.
 *  - Return value: SS_OK (0) or a negative SS_ERR_* code.  Argument errors
 *    are detected before any work is enqueued; ss_last_error() returns a
 *    thread-local message for the last failing call.
 *  - Data problems of one object never fail a call: they are reported in
 *    obj_status[] (SS_OBJ_*), that object's periodogram row is NaN, its
 *    best index is -1 and its best period/power are NaN.
 *  - A context is not thread-safe; use one context per host thread.
 */
#ifndef SSGPU_H
#define SSGPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes */
#define SS_OK 0
#define SS_ERR_INVALID_ARG (-1) /* null pointer, bad size, bad grid/span/precision */
#define SS_ERR_HIP (-2)         /* a HIP runtime call failed (message has the hipError text) */
#define SS_ERR_OOM (-3)         /* workspace allocation failed */
#define SS_ERR_UNSUPPORTED (-4) /* e.g. an object longer than SS_MAX_POINTS */
#define SS_ERR_INVARIANT (-5)   /* debug mode: an invariant check failed (message has the counts) */

/* ---- per-object status (obj_status[]) */
#define SS_OBJ_OK 0
#define SS_OBJ_TOO_FEW 1    /* fewer than 5 points */
#define SS_OBJ_BAD_ERR 2    /* an error bar e <= 0 or non-finite */
#define SS_OBJ_NONFINITE 3  /* a non-finite t or y */
#define SS_OBJ_CONST_MAG 4  /* chi0 == 0: constant magnitudes */
#define SS_OBJ_TOO_LONG 5   /* more than SS_MAX_POINTS points, or too long for the
                               LDS of one trial group at the requested spans */
#define SS_OBJ_BAD_RANGE 6  /* its offsets are decreasing or fall outside [0, n_points] */
/* Precedence when several apply: BAD_RANGE, TOO_FEW, NONFINITE, BAD_ERR, CONST_MAG,
 * TOO_LONG. */

/* ---- precision (ss_params.precision) */
#define SS_FP64 0  /* every sum and fit in FP64; periodogram is double */
#define SS_FP32C 1 /* FP32 arithmetic with compensated (two-float) window sums;
                      FP64 fold and chi^2/chi0 normalisation; periodogram is float.
                      The precision study: on MI355X FP64 runs at the unpacked FP32
                      rate, and SS_FP64 is the faster and production path */

/* ---- method (ss_best_period, ss_method_periodogram) */
#define SS_METHOD_SS 0      /* Listing 1: cross-validated variable-span smoother */
#define SS_METHOD_SSSP 1    /* Sec. 3: single-pass generalized validation, read as one
                               sweep over the three spans with GCV_k = RSS_k / (1 -
                               TR_k/n)^2 choosing one span per trial (first minimum),
                               chi^2 = RSS of that span */
#define SS_METHOD_SSSP_GV 2 /* Sec. 3, second reading: the same sweep, then a span per
                               point by |y - s_k| / (1 - TR_k/n) (Listing 1's scan:
                               strict <, from 1e20), bass enhancement against the
                               largest span, clip and blend as in Listing 1, chi^2 of
                               the blend (no residual, span or final smooth) */

/* Largest light curve the library accepts (points per object).  On MI355X
 * (160 KB of LDS per workgroup) a trial group for more than 3,072 points does not
 * fit at any span_max >= 0.1, so such objects are reported SS_OBJ_TOO_LONG; up to
 * 3,072 points run at the default spans. */
#define SS_MAX_POINTS 4096

typedef struct ss_ctx ss_ctx;

/* Trial frequencies f_k = f_min + k*df, df = (f_max - f_min)/n_freq,
 * k = 0 .. n_freq-1: the even grid on [f_min, f_max) of App. A / Alg. 1.
 * Requires 0 < f_min < f_max and n_freq >= 1. */
typedef struct {
    double f_min;
    double f_max;
    int64_t n_freq;
} ss_grid;

/* Smoother parameters.  span_min/mid/max are the tweeter, midrange and woofer
 * spans of Listing 1 (defaults 0.05, 0.2, 0.5; need 0 < min < mid < max <= 1).
 * alpha is the bass-enhancement exponent (Listing 1: applied when
 * 0 < alpha <= 10; default 9, the paper's choice for catalogs, Sec. 5.1).
 * fixed_span > 0 replaces the variable span by one smooth at that span
 * (Listing 1's fixed-span branch; for the single-pass variant it leaves one
 * candidate span).  flags: 0, or the debug bits below (full-grid calls only:
 * the periodogram calls and ss_best_period; the other calls reject them). */
typedef struct {
    double span_min;
    double span_mid;
    double span_max;
    double alpha;
    double fixed_span;
    int32_t precision;
    int32_t flags;
} ss_params;

/* Debug mode.  SS_FLAG_CHECK_INVARIANTS: after the trials, the call re-runs
 * the trial kernels' fold and sort (Sec. 2.2) and their window sums
 * (Listing 1's running-line windows) over the same work items and checks
 * that the sorted phases increase (keys of equal phase in point order) and
 * that every window of a used span has a positive weight sum W; it then
 * waits for the device, keeps the counts (ss_ctx_check_counts) and returns
 * SS_ERR_INVARIANT if anything is wrong.  Results are those of the call
 * without the flag.  SS_FLAG_CHECK_SELFTEST (with the first) inverts the
 * order test, so that every trial of two or more points is reported: a test
 * that the check reports. */
#define SS_FLAG_CHECK_INVARIANTS 1
#define SS_FLAG_CHECK_SELFTEST 2

/* A catalog of light curves in CSR form (device memory, FP64):
 * object o owns points offsets[o] .. offsets[o+1]-1 of t (days), y
 * (magnitudes) and e (error bars); offsets has n_obj+1 entries and n_points
 * is the length of t, y and e (normally offsets[n_obj]).  The library sizes
 * its workspace from n_points and never reads offsets on the host.  Points
 * need not be time-sorted. */
typedef struct {
    int64_t n_obj;
    int64_t n_points;
    const int64_t *offsets;
    const double *t;
    const double *y;
    const double *e;
} ss_catalog;

/* Fills *p with the defaults above (FP64). */
void ss_params_default(ss_params *p);

/* Creates a context bound to HIP device `device`.  The context owns a
 * workspace that grows on demand and is freed by ss_ctx_destroy. */
int ss_ctx_create(int device, ss_ctx **out);
void ss_ctx_destroy(ss_ctx *ctx);

/* Periodogram of the Super Smoother (Alg. 1 with Listing 1):
 * pgram[o*n_freq + k] = 1 - chi2(o, f_k)/chi0(o), where chi2 is the weighted
 * residual sum of the smoothed phase curve and chi0 the weighted sum of
 * squares about the weighted mean.  pgram is double (SS_FP64) or float
 * (SS_FP32C), n_obj*n_freq entries; obj_status has n_obj entries. */
int ss_periodogram(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                   const ss_params *params, void *pgram, int32_t *obj_status, void *stream);

/* Same for the single-pass generalized-validation variant (Sec. 3): per trial
 * the candidate span with the smallest GCV = RSS/(1 - TR/n)^2 is kept and
 * chi2 = its RSS.  params.alpha is ignored. */
int sssp_periodogram(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                     const ss_params *params, void *pgram, int32_t *obj_status, void *stream);

/* Periodogram of any method (SS_METHOD_*): as ss_periodogram, with the method
 * chosen by `method` (alpha used by SS and SSSP_GV). */
int ss_method_periodogram(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                          const ss_grid *grid, const ss_params *params, void *pgram,
                          int32_t *obj_status, void *stream);

/* Two finders from one fold and sort: the method's periodogram (as
 * ss_method_periodogram) and, from the same sorted phases of every trial, the
 * phase-dispersion periodogram pgram_pdm [n_obj * n_freq] (same type): the
 * fraction of chi0 explained by the weighted means of n_bins equal phase bins
 * (bin b holds the points with b <= B phase < b + 1, phase from the FP64 fold
 * as a 48-bit fixed-point value), i.e. sum_b (sum w (y - ybar))^2 / (sum w)
 * / chi0.  n_bins = 0 uses clamp(n / 5, 4, 32) per object; else 2..256.
 * Bad objects get NaN rows in both. */
int ss_pdm_periodogram(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                       const ss_grid *grid, const ss_params *params, int32_t n_bins,
                       void *pgram, void *pgram_pdm, int32_t *obj_status, void *stream);

/* Best period per object without materialising the periodogram (Alg. 1
 * findPeriod): best_idx[o] = the lowest k attaining the largest P (NaN
 * skipped), best_period[o] = 1/f_k, best_power[o] = that P (as double).
 * method = SS_METHOD_SS or SS_METHOD_SSSP.  Each output has n_obj entries. */
int ss_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat, const ss_grid *grid,
                   const ss_params *params, int64_t *best_idx, double *best_period,
                   double *best_power, int32_t *obj_status, void *stream);

/* ---- shared time sampling
 *
 * Objects observed at the same times (a survey field imaged together) fold
 * and sort alike at every trial frequency (Sec. 2.2: the fold and the sort
 * depend only on the times).  A shared catalog holds n_obj light curves of
 * n_points each at the times t[n_points] (device, FP64, need not be sorted);
 * y and e are device FP64 arrays [n_obj][n_points], object-major.  The
 * library folds and sorts once per trial frequency for a batch of objects
 * and runs the smoother of each object on that order.  Results, statuses and
 * errors are those of ss_method_periodogram / ss_best_period on the same
 * objects written as an ordinary catalog (offsets o * n_points, t repeated),
 * except that a non-finite time gives every object SS_OBJ_NONFINITE. */
typedef struct {
    int64_t n_obj;
    int64_t n_points;
    const double *t; /* [n_points] */
    const double *y; /* [n_obj][n_points] */
    const double *e; /* [n_obj][n_points] */
} ss_shared_catalog;

int ss_shared_periodogram(ss_ctx *ctx, int32_t method, const ss_shared_catalog *cat,
                          const ss_grid *grid, const ss_params *params, void *pgram,
                          int32_t *obj_status, void *stream);
int ss_shared_best_period(ss_ctx *ctx, int32_t method, const ss_shared_catalog *cat,
                          const ss_grid *grid, const ss_params *params, int64_t *best_idx,
                          double *best_period, double *best_power, int32_t *obj_status,
                          void *stream);

/* ---- memory planning and batched periodograms
 *
 * Sec. 4.1, Eq. 1 splits a search into N_b = r (beta s)^-1 batches, r being
 * the estimated device footprint, s the device memory and beta = 0.75 a
 * safety factor.  The fused kernels here keep no N_f x N_t scratch; what
 * grows with a catalog is the periodogram itself (n_obj x n_freq values,
 * 200 GB for a million objects x 50,000 frequencies in FP32).
 * ss_plan_batches applies Eq. 1 to that footprint, r = fixed + n_obj * per,
 * with fixed = 32 bytes per point of prep workspace and per = the output row
 * (if want_pgram) + the per-tile partials + per-object arrays, and splits the
 * objects: *objs_per_batch = floor((beta s - fixed) / per) (at most n_obj),
 * *n_batches = ceil(n_obj / *objs_per_batch).  s = mem_bytes, or the
 * device's free memory when mem_bytes = 0.  SS_ERR_OOM if not one object
 * fits.
 *
 * ss_periodogram_batched computes the periodogram of a catalog in object
 * batches of chunk_objs into the caller's device buffer `chunk`
 * (chunk_objs x n_freq values of the precision's type) and after each batch
 * waits for `stream` and calls sink(user, obj_begin, obj_end, chunk,
 * obj_status + obj_begin) on the calling thread; the sink must take what it
 * needs before returning (the next batch overwrites chunk).  Rows and
 * statuses are those of ss_method_periodogram on the whole catalog. */
typedef void (*ss_pgram_sink)(void *user, int64_t obj_begin, int64_t obj_end, const void *chunk,
                              const int32_t *obj_status);
int ss_plan_batches(ss_ctx *ctx, int64_t n_obj, int64_t n_points, const ss_grid *grid,
                    int32_t precision, int32_t want_pgram, double beta, int64_t mem_bytes,
                    int64_t *objs_per_batch, int64_t *n_batches);
int ss_periodogram_batched(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, void *chunk,
                           int64_t chunk_objs, ss_pgram_sink sink, void *user,
                           int32_t *obj_status, void *stream);

/* Allocation-free best period, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, hosts that
 * forbid allocation): ss_best_period computed in a fixed device region of
 * SS_NOALLOC_BYTES that the library holds on every device it runs on until
 * the process ends, instead of the context's growing workspace.  The call
 * makes no hipMalloc or hipFree; the caller still passes the outputs.
 * Needed: 32 bytes per point, 72 per object and 12 per object and frequency
 * tile (tiles as chosen by ss_ctx_set_tile or automatically), each part
 * rounded up to 256 bytes; a catalog that needs more than SS_NOALLOC_BYTES
 * gets SS_ERR_UNSUPPORTED before any work is queued.  The size classes of a
 * catalog run one after another on `stream` (not forked).  Every call on a
 * device shares that device's region and leaves its contents behind: calls
 * that overlap in time on one device (other streams, other threads, other
 * contexts) race and give wrong results. */
#define SS_NOALLOC_BYTES (64ll << 20)
int ss_best_period_noalloc(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, int64_t *best_idx,
                           double *best_period, double *best_power, int32_t *obj_status,
                           void *stream);

/* Trial-group shapes (autotuning).  One trial runs on a workgroup of `nw`
 * wavefronts whose threads hold `ppl` consecutive phase-sorted points each,
 * so a shape holds light curves of up to 64*nw*ppl points.  ss_num_shapes /
 * ss_shape_info list the shapes the library is built with.
 * ss_ctx_set_shape(ctx, n_max, nw, ppl) adds a rule: objects with
 * n <= n_max (and above the n_max of every smaller rule) run on that shape;
 * objects no rule covers use the built-in default.  nw = 0 clears every rule.
 * Returns SS_ERR_UNSUPPORTED for a shape that is not built in or holds fewer
 * than n_max points.  ss_ctx_set_tile sets the number of trial frequencies
 * per work item (0 = automatic). */
int ss_num_shapes(void);
int ss_shape_info(int index, int32_t *nw, int32_t *ppl);
int ss_ctx_set_shape(ss_ctx *ctx, int32_t n_max, int32_t nw, int32_t ppl);
int ss_ctx_set_tile(ss_ctx *ctx, int32_t tile_f);

/* Whether the size classes of one call run concurrently (enable != 0:
 * launches forked onto internal streams and joined back to the call's
 * stream) or one after another on the call's stream (0, the default, which
 * measured faster on MI355X). */
int ss_ctx_set_concurrency(ss_ctx *ctx, int32_t enable);

/* Kernel timing, for benchmarks.  With timing enabled, every call records HIP
 * events on its stream around each launch of the fused trial kernel; when
 * concurrency is on (ss_ctx_set_concurrency) and a call has several size
 * classes, one pair of events spans the fork to the join.  ss_ctx_trial_kernel_ms waits for the last call's events and
 * returns the summed duration of its trial-kernel launches in milliseconds
 * and their count.  Returns SS_ERR_INVALID_ARG if timing was off. */
int ss_ctx_set_timing(ss_ctx *ctx, int enable);
int ss_ctx_trial_kernel_ms(ss_ctx *ctx, double *ms, int32_t *n_launches);

/* ---- learned frequency proposal + exact refine (search-and-refine, Sec. 6)
 *
 * A set encoder ranks 1024 log-spaced frequency bins of the search grid for
 * each object; the exact Super Smoother (or SSSP) trial kernel then searches
 * only the fine-grid frequencies inside the top bins.  The full-grid search
 * (ss_best_period) stays the reference: a refined result is the full-grid
 * result whenever the full-grid best frequency lies in the refined set.
 *
 * Bins: bin b holds the grid indices k with E_b <= f_k < E_{b+1}, where
 * E_b = f_min * (f_max / f_min)^(b / 1024) in FP64 (b = 0..1024), f_k as in
 * ss_grid.  ss_bin_table writes the first index of each bin (and n_freq as
 * entry 1024) to a HOST array of 1025 int64; it needs no device.
 *
 * Network (SS_ENC_PARAMS FP32 parameters, flat, row-major, input dimension
 * first): W1[80][64], W2[64][128], b2[128], W3[128][1024], b3[1024].
 * Per point i of an object: features x_i[80] = sin and cos of 2 pi g_m tt_i
 * (slots 2m, 2m+1; g_m = 32 frequencies log-spaced over [f_min, f_max], ends
 * included), (y_i - ybar)/sigma (slot 64), e_i/sigma (slot 65) and 1 (slot
 * 66; row 66 of W1 is the first layer's bias), other slots 0; ybar is the
 * e^-2-weighted mean, sigma^2 = chi0 / sum(e^-2), tt = t - min t.  Then
 * h1 = relu(x W1), h2 = relu(h1 W2 + b2), emb = mean over points of h2,
 * logits = emb W3 + b3.  The per-point layers run in BF16 on the matrix
 * cores with FP32 accumulation; the head, the loss and Adam run in FP32.
 * Objects with a nonzero status get emb = 0 (logits = b3) and no refine.
 */
#define SS_ENC_PARAMS 145536
#define SS_ENC_BINS 1024

/* First grid index of each log bin (host output, 1025 entries). */
int ss_bin_table(const ss_grid *grid, int64_t *first_k);

/* Number of encoder parameters (SS_ENC_PARAMS). */
int ss_enc_num_params(void);

/* Encoder forward: emb [n_obj][128] and logits [n_obj][1024] (device FP32),
 * feature frequencies and bins from `grid`; obj_status as in ss_best_period. */
int ss_enc_forward(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                   const float *enc_params, float *emb, float *logits, int32_t *obj_status,
                   void *stream);

/* Training gradient: mean softmax cross-entropy of the logits against
 * labels[n_obj] (bin indices; objects with a label outside [0, 1024) or a
 * nonzero status contribute 0 but still count in the mean), written to
 * *loss (device float), and its gradient with respect to every parameter
 * (grad: device, SS_ENC_PARAMS floats, overwritten).  Deterministic for a
 * given device and catalog.  Needs n_obj >= 1. */
int ss_enc_train_grad(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid,
                      const float *enc_params, const int32_t *labels, float *grad, float *loss,
                      int32_t *obj_status, void *stream);

/* One Adam step on FP32 master weights, in place: m = b1 m + (1-b1) g,
 * v = b2 v + (1-b2) g^2, p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * step counts from 1.  All arrays are device, n floats. */
int ss_adam_step(float *params, const float *grad, float *m, float *v, int64_t n, int32_t step,
                 float lr, float beta1, float beta2, float eps, void *stream);

/* Refine from given logits [n_obj][1024] (device FP32): per object the top_k
 * bins by logit (NaN ranks lowest; equal logits: lower bin first), each
 * widened by `margin` bins on both sides, are searched at every grid
 * frequency they hold, and the best over that set is reported exactly as
 * ss_best_period reports it (lowest index among equal powers).  Objects with
 * fewer than full_below points are searched on the whole grid instead (0 =
 * never).  1 <= top_k <= 1024, 0 <= margin <= 64, full_below >= 0. */
int ss_refine_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                          const ss_grid *grid, const ss_params *params, const float *logits,
                          int32_t top_k, int32_t margin, int32_t full_below, int64_t *best_idx,
                          double *best_period, double *best_power, int32_t *obj_status,
                          void *stream);

/* Cheap exact-grid proposal scores [n_obj][1024] (device FP32): for every grid
 * frequency, the light curve is folded (FP64 phase, as for the trials) into
 * B = clamp(n / 5, 4, 32) equal phase bins and scored by the fraction of chi0
 * explained by the bins' weighted means, sum_b (sum_{i in b} w_i yc_i)^2 /
 * (sum_{i in b} w_i) / chi0 with yc = y - ybar (FP32 sums, FP64 phase and
 * bin index); each log bin gets the maximum over its grid frequencies (0 if
 * it holds none; all 0 for objects with a nonzero status).  A phase-
 * dispersion statistic: no sort, no smoother. */
int ss_bin_scores(ss_ctx *ctx, const ss_catalog *cat, const ss_grid *grid, float *scores,
                  int32_t *obj_status, void *stream);

/* Proposal + exact refine in one call.  The bins are ranked by
 * logit_b + gamma * score_b, where logit_b comes from the encoder
 * (enc_params; NULL = no encoder, logits 0) and score_b from ss_bin_scores
 * (gamma = 0: not computed).  gamma >= 0; at least one of the two terms must
 * be present.  top_k, margin and full_below as for ss_refine_best_period.
 * The first call on a new grid uploads the bin table synchronously. */
int ss_learned_best_period(ss_ctx *ctx, int32_t method, const ss_catalog *cat,
                           const ss_grid *grid, const ss_params *params, const float *enc_params,
                           float gamma, int32_t top_k, int32_t margin, int32_t full_below,
                           int64_t *best_idx, double *best_period, double *best_power,
                           int32_t *obj_status, void *stream);

/* ---- model object: a proposal network bound to one search grid
 *
 * The learned half of search-and-refine (Sec. 6) as one object: the encoder's
 * SS_ENC_PARAMS FP32 master parameters (layout above), its Adam moments
 * m and v, the Adam step count and hyper-parameters (beta1 0.9, beta2 0.999,
 * eps 1e-8), and the grid it was trained for (its bins and feature
 * frequencies follow from the grid).  The model lives on the device of the
 * context that created or loaded it; it is not thread-safe.
 *
 * File format (ss_model_save / ss_model_load), little-endian:
 *   bytes 0..7    "SSGPUMDL"
 *   uint32        format version (1)
 *   uint32        J = length of the JSON metadata
 *   uint64        n_params; int32 step; float32 beta1, beta2, eps;
 *   float64       f_min, f_max; int64 n_freq; uint64 array offset A
 *   J bytes       JSON metadata (format, versions, layer layout, grid, bin
 *                 rule, the 32 feature frequencies, step, Adam settings)
 *   at byte A     float32 params[n_params], m[n_params], v[n_params]
 * Loading checks the magic, the format version, n_params, the grid and the
 * file length; the JSON is for readers and is not parsed. */
typedef struct ss_model ss_model;

/* New model for `grid` with parameters copied from the HOST array
 * init_params[SS_ENC_PARAMS]; Adam state zero, step 0.  Synchronous. */
int ss_model_create(ss_ctx *ctx, const ss_grid *grid, const float *init_params,
                    ss_model **out);
void ss_model_destroy(ss_model *model);

/* Any of grid, step, device_params may be NULL.  *device_params points at
 * the model's current parameters (device, SS_ENC_PARAMS floats, owned by the
 * model; valid until ss_model_destroy). */
int ss_model_info(const ss_model *model, ss_grid *grid, int32_t *step,
                  const float **device_params);

/* Copies the model's current parameters to dst (device, SS_ENC_PARAMS
 * floats), asynchronously on `stream`. */
int ss_model_copy_params(const ss_model *model, float *dst, void *stream);

/* Writes the model to `path` (format above).  Waits for the model's device
 * first, so that queued training steps are included.  Errors: SS_ERR_HIP,
 * SS_ERR_INVALID_ARG when the file cannot be written. */
int ss_model_save(const ss_model *model, const char *path);

/* Reads a model written by ss_model_save onto ctx's device (synchronous).
 * SS_ERR_INVALID_ARG for a missing, truncated or malformed file,
 * SS_ERR_UNSUPPORTED for another format version. */
int ss_model_load(ss_ctx *ctx, const char *path, ss_model **out);

/* The file format on the host alone (no device): write / read the grid,
 * the step count and HOST arrays params, adam_m, adam_v of SS_ENC_PARAMS
 * floats each.  Errors as for ss_model_save / ss_model_load; a file whose
 * Adam settings differ from the fixed ones above is rejected. */
int ss_model_file_write(const char *path, const ss_grid *grid, int32_t step,
                        const float *params, const float *adam_m, const float *adam_v);
int ss_model_file_read(const char *path, ss_grid *grid, int32_t *step, float *params,
                       float *adam_m, float *adam_v);

/* One training step: the mean cross-entropy gradient of the batch
 * (as ss_enc_train_grad on the model's grid; labels[n_obj] device int32,
 * *loss device float) followed by one Adam step with learning rate lr on the
 * model's parameters and moments; the model's step count goes up by one.
 * Asynchronous on `stream`. */
int ss_train_step(ss_ctx *ctx, ss_model *model, const ss_catalog *batch, const int32_t *labels,
                  float lr, float *loss, int32_t *obj_status, void *stream);

/* Search-and-refine with a model: ss_learned_best_period with the model's
 * parameters.  `grid` must be the grid the model was made for
 * (SS_ERR_INVALID_ARG otherwise). */
int ss_best_period_learned(ss_ctx *ctx, const ss_model *model, int32_t method,
                           const ss_catalog *cat, const ss_grid *grid, const ss_params *params,
                           float gamma, int32_t top_k, int32_t margin, int32_t full_below,
                           int64_t *best_idx, double *best_period, double *best_power,
                           int32_t *obj_status, void *stream);

/* Message for the last failing call on this host thread ("" if none). */
const char *ss_last_error(void);

/* ABI version (major*100 + minor). */
int ss_version(void);

/* Counts of the last call made with SS_FLAG_CHECK_INVARIANTS on this
 * context: out[0] trials checked, out[1] adjacent sorted keys out of order,
 * out[2] windows with W <= 0 (all 0 before such a call).  Host memory. */
int ss_ctx_check_counts(ss_ctx *ctx, int64_t *out);

#ifdef __cplusplus
}
#endif

#endif /* SSGPU_H */
