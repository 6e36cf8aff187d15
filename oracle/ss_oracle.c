/*
 * ss_oracle.c -- CPU oracle for the Super Smoother period search.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * FP64 statement of what the GPU path computes.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it.  It
 * shares no code, header, table or helper with the HIP library, and the HIP
 * library never calls it.
 *
 * Source: Gowanlock, Butler, Trilling & McNeill, "GPU-Enabled Searches for
 * Periodic Signals of Unknown Shape" (arXiv 2111.07396).  Citations below name
 * the paper's section, algorithm, listing or equation.
 *
 * What each function follows:
 *   ora_prep        Alg. 1 step compute_chi0_tt_weights (Sec. 2.2): w = e^-2,
 *                   tt = t - min(t); chi0 read as the weighted sum of squares
 *                   about the weighted mean (the paper names chi0 but prints no
 *                   formula).
 *   ora_freq        Sec. 2.2 findPeriod and App. A: even grid on [fmin, fmax),
 *                   f_k = fmin + k*df, df = (fmax - fmin)/n_freq.
 *   ora_fold        Sec. 2.2: t1 = (tt mod p)/p with p = 1/f.
 *   ora_argsort     Sec. 2.2: stable argsort by phase (ties keep time order).
 *   ora_smooth      The running-line smoother that Listing 1 calls (Friedman
 *                   1984, cited in Sec. 2.2; the body is not printed in the
 *                   paper).  Written here as its definition: for every point a
 *                   weighted least-squares line over an explicit window,
 *                   computed directly with two passes over that window.
 *   ora_supsmu      The variable-span Super Smoother that Sec. 2.2 runs per
 *                   trial, written from the method: primary fits and their
 *                   cross-validation errors per candidate span, a span per
 *                   point (least error, bass enhancement), the spans
 *                   smoothed, the fits mixed at them, a final smooth.
 *   ora_sssp        Sec. 3 single-pass generalized-validation variant.  The
 *                   paper gives no equation; the reading implemented is one
 *                   sweep over K candidate spans scored by generalized
 *                   cross-validation GCV_k = RSS_k / (1 - TR_k/n)^2, the first
 *                   minimum wins, chi^2 = RSS_k*.
 *   ora_sssp2       A second reading of the Sec. 3 variant: the same single
 *                   sweep (smooths s_k and traces TR_k of the K = 3 spans),
 *                   then a span choice per point by the un-smoothed
 *                   generalized-validation residual |y - s_k| / (1 - TR_k/n)
 *                   with the Super Smoother's per-point span selection and
 *                   mixing of fits (its error, span and final smooths left
 *                   out).
 *   ora_pdm         Phase dispersion of one trial (a second period finder on the
 *                   same fold; Sec. 6 names reusing the fold and sort for other
 *                   finders): the points' phases in B equal bins, the fraction
 *                   of chi0 explained by the bins' weighted means.
 *   ora_trial       fold -> sort -> smoother -> chi^2 -> P = 1 - chi^2/chi0
 *                   (Alg. 1 computePgram; formula read as stated).
 *   ora_periodogram Alg. 1 over a catalog of objects (Sec. 4.3 batch mode).
 *   ora_best        Alg. 1 findPeriod: argmax of P (lowest index on ties, NaN
 *                   skipped), period = 1/(fmin + x*df).
 *
 * Parity status: every function above is pinned by the tests against brute
 * force, closed forms, textbook special cases, invariants or numbers printed
 * in the paper (Table 2 grid sizes).  None is "parity unpinned".
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared (see build.sh).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_TOO_FEW 1
#define ORA_BAD_ERR 2
#define ORA_NONFINITE 3
#define ORA_CONST_MAG 4

#define ORA_METHOD_SS 0
#define ORA_METHOD_SSSP 1
#define ORA_METHOD_SSSP2 2

/* ------------------------------------------------------------------ prep */

/* Alg. 1, compute_chi0_tt_weights.  Returns a per-object status; the outputs
 * are written only when the status is ORA_OK.  Status precedence: too few
 * points (n < 5; the listing's quartile scale needs n >= 4 and the smallest
 * window needs 5 points), non-finite t or y, bad error bar (e <= 0 or
 * non-finite), zero chi0. */
int ora_prep(int64_t n, const double *t, const double *y, const double *e,
             double *tt, double *w, double *ybar_out, double *chi0_out)
{
    if (n < 5) return ORA_TOO_FEW;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(t[i]) || !isfinite(y[i])) return ORA_NONFINITE;
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(e[i]) || !(e[i] > 0.0)) return ORA_BAD_ERR;
    double tmin = t[0];
    for (int64_t i = 1; i < n; ++i)
        if (t[i] < tmin) tmin = t[i];
    double sw = 0.0, swy = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = 1.0 / (e[i] * e[i]);
        sw += wi;
        swy += wi * y[i];
    }
    double ybar = swy / sw;
    double chi0 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double wi = 1.0 / (e[i] * e[i]);
        double d = y[i] - ybar;
        chi0 += wi * d * d;
    }
    if (!(chi0 > 0.0)) return ORA_CONST_MAG;
    for (int64_t i = 0; i < n; ++i) {
        tt[i] = t[i] - tmin;
        w[i] = 1.0 / (e[i] * e[i]);
    }
    if (ybar_out) *ybar_out = ybar;
    if (chi0_out) *chi0_out = chi0;
    return ORA_OK;
}

/* ------------------------------------------------------------------ grid */

double ora_freq(double fmin, double fmax, int64_t n_freq, int64_t k)
{
    double df = (fmax - fmin) / (double)n_freq;
    double kd = (double)k;
    double step = kd * df;
    return fmin + step;
}

/* Sec. 5.3: grid spacing 0.1/T_max and N_f = (fmax - fmin)/df (Table 2). */
int64_t ora_grid_nfreq(double t_extent_max, double fmin, double fmax)
{
    double df = 0.1 / t_extent_max;
    return (int64_t)floor((fmax - fmin) / df + 0.5);
}

/* ------------------------------------------------------------------ fold + sort */

void ora_fold(int64_t n, const double *tt, double f, double *phase)
{
    double p = 1.0 / f;
    for (int64_t i = 0; i < n; ++i) phase[i] = fmod(tt[i], p) / p;
}

typedef struct {
    double key;
    int64_t idx;
} ora_pair;

static int cmp_pair(const void *a, const void *b)
{
    const ora_pair *pa = (const ora_pair *)a, *pb = (const ora_pair *)b;
    if (pa->key < pb->key) return -1;
    if (pa->key > pb->key) return 1;
    if (pa->idx < pb->idx) return -1;
    if (pa->idx > pb->idx) return 1;
    return 0;
}

/* Stable argsort: order by phase, equal phases keep their input order.  The
 * library sort is made stable by comparing the original index second. */
void ora_argsort(int64_t n, const double *key, int64_t *perm)
{
    ora_pair *p = (ora_pair *)malloc((size_t)n * sizeof(ora_pair));
    for (int64_t i = 0; i < n; ++i) {
        p[i].key = key[i];
        p[i].idx = i;
    }
    qsort(p, (size_t)n, sizeof(ora_pair), cmp_pair);
    for (int64_t i = 0; i < n; ++i) perm[i] = p[i].idx;
    free(p);
}

/* ------------------------------------------------------------------ smoother */

/* Half-width of the running-line window for a span: b = max(2, floor(span*n/2
 * + 1/2)); clamped so a window never holds a point twice (2b+1 <= n). */
int ora_halfwidth(int n, double span)
{
    int b = (int)(0.5 * span * (double)n + 0.5);
    if (b < 2) b = 2;
    if (2 * b + 1 > n) b = (n - 1) / 2;
    return b;
}

/* Window members of point j: index and the phase shift applied to x.
 * Periodic: the 2b+1 cyclic neighbours j-b .. j+b; a neighbour taken from the
 * other end of the cycle has its x moved by -1 (left) or +1 (right).
 * Non-periodic: the 2b+1 consecutive points starting at
 * lo = clamp(j-b, 0, n-1-2b). */
static void window_member(int n, int j, int b, int periodic, int m, int *idx, double *shift)
{
    if (periodic) {
        int i = j - b + m;
        if (i < 0) {
            *idx = i + n;
            *shift = -1.0;
        } else if (i >= n) {
            *idx = i - n;
            *shift = 1.0;
        } else {
            *idx = i;
            *shift = 0.0;
        }
    } else {
        int lo = j - b;
        if (lo < 0) lo = 0;
        if (lo > n - 1 - 2 * b) lo = n - 1 - 2 * b;
        *idx = lo + m;
        *shift = 0.0;
    }
}

/* The running-line smoother S(x, v, w, span) on x sorted ascending.
 *   s[j]   = weighted least-squares line of (x, v) over the window of j,
 *            evaluated at x[j]; the slope is dropped (s = window mean of v)
 *            when the window's weighted sum of squared x-deviations V is not
 *            above vsmlsq.
 *   r[j]   (cv != 0) = |v[j] - s[j]| / (1 - w[j]*h[j]) with
 *            h[j] = 1/W + (x[j]-xbar)^2/V (second term only when V > vsmlsq),
 *            the leave-one-out residual; when 1 - w h <= 0 it repeats r[j-1]
 *            (0 for j = 0).  r uses s before tie averaging.
 *   lev[j] (optional) = h[j] as above.
 * Finally s is replaced, over every run of equal x (x[j+1] <= x[j]), by the
 * run's weighted mean of s. */
void ora_smooth(int n, const double *x, const double *v, const double *w, double span,
                int periodic, int cv, double vsmlsq, double *s, double *r, double *lev)
{
    int b = ora_halfwidth(n, span);
    int m = 2 * b + 1;
    for (int j = 0; j < n; ++j) {
        double W = 0.0, Sx = 0.0, Sv = 0.0;
        for (int q = 0; q < m; ++q) {
            int i;
            double sh;
            window_member(n, j, b, periodic, q, &i, &sh);
            W += w[i];
            Sx += w[i] * (x[i] + sh);
            Sv += w[i] * v[i];
        }
        double xm = Sx / W, vm = Sv / W;
        double V = 0.0, C = 0.0;
        for (int q = 0; q < m; ++q) {
            int i;
            double sh;
            window_member(n, j, b, periodic, q, &i, &sh);
            double dx = (x[i] + sh) - xm;
            V += w[i] * dx * dx;
            C += w[i] * dx * (v[i] - vm);
        }
        double slope = (V > vsmlsq) ? C / V : 0.0;
        double dxj = x[j] - xm;
        s[j] = vm + slope * dxj;
        double h = 1.0 / W;
        if (V > vsmlsq) h += dxj * dxj / V;
        if (lev) lev[j] = h;
        if (cv) {
            double d = 1.0 - w[j] * h;
            if (d > 0.0)
                r[j] = fabs(v[j] - s[j]) / d;
            else
                r[j] = (j > 0) ? r[j - 1] : 0.0;
        }
    }
    /* tie averaging */
    int j = 0;
    while (j < n) {
        int j0 = j;
        double sws = w[j] * s[j], sw = w[j];
        while (j + 1 < n && x[j + 1] <= x[j]) {
            ++j;
            sws += w[j] * s[j];
            sw += w[j];
        }
        if (j > j0) {
            double a = (sw > 0.0) ? sws / sw : 0.0;
            for (int i = j0; i <= j; ++i) s[i] = a;
        }
        ++j;
    }
}

/* ------------------------------------------------------------------ trial frame */

/* What every smooth of one trial shares: the sorted abscissae and weights,
 * the mode and the threshold below which a window's x-spread counts as zero. */
typedef struct {
    int n;
    const double *x, *w;
    int periodic;
    double vsmlsq;
} ora_frame;

/* Sec. 2.2: when the sorted phases do not spread (last <= first) the fit is
 * the weighted mean of y at every point.  Returns 1 and fills fit then. */
static int flat_phases(int n, const double *x, const double *y, const double *w, double *fit)
{
    if (x[n - 1] > x[0]) return 0;
    double num = 0.0, den = 0.0;
    for (int j = 0; j < n; ++j) {
        num += w[j] * y[j];
        den += w[j];
    }
    const double mean = (den > 0.0) ? num / den : 0.0;
    for (int j = 0; j < n; ++j) fit[j] = mean;
    return 1;
}

/* Sec. 2.2: the zero-spread threshold is 1e-6 times the squared distance
 * between the sorted abscissae of 1-based ranks q and 3q, q = floor(n/4)
 * (lower and upper quartile points; no widening when it is 0). */
static double zero_spread(int n, const double *x)
{
    const int q = n / 4;
    const double d = x[3 * q - 1] - x[q - 1];
    return 1.0e-6 * d * d;
}

/* iper = 2 asks for the periodic mode, granted when every abscissa lies in
 * [0, 1] (always so for phases); iper = 1 is the plain mode. */
static ora_frame make_frame(int n, const double *x, const double *w, int iper)
{
    ora_frame F;
    F.n = n;
    F.x = x;
    F.w = w;
    F.periodic = (iper == 2) && x[0] >= 0.0 && x[n - 1] <= 1.0;
    F.vsmlsq = zero_spread(n, x);
    return F;
}

static void frame_smooth(const ora_frame *F, const double *v, double span, int cv, double *s,
                         double *r, double *lev)
{
    ora_smooth(F->n, F->x, v, F->w, span, F->periodic, cv, F->vsmlsq, s, r, lev);
}

/* ------------------------------------------------------------------ per-point span selection */

/* Cross-validation errors at or above this value never select a span. */
#define ORA_ERR_CAP 1.0e20

/* Index of the candidate span with the least error at one point (spans in
 * ascending order, the smaller one kept on equal errors); -1 when no error is
 * below ORA_ERR_CAP (or all are NaN).  *least receives that error (the cap
 * when none). */
static int least_error(const double err[3], double *least)
{
    int k_best = -1;
    double e_best = ORA_ERR_CAP;
    for (int k = 0; k < 3; ++k) {
        if (err[k] < e_best) {
            e_best = err[k];
            k_best = k;
        }
    }
    *least = e_best;
    return k_best;
}

/* Bass enhancement (Sec. 2.2): with 0 < alpha <= 10, a span chosen at a point
 * whose least error e is positive and below the woofer's error e_w moves
 * toward the woofer span by the fraction max(e/e_w, 1e-7)^(10 - alpha). */
static double bass_shift(double span, double e, double e_w, double woofer, double alpha)
{
    if (!(alpha > 0.0 && alpha <= 10.0)) return span;
    if (!(e > 0.0 && e < e_w)) return span;
    double ratio = e / e_w;
    if (ratio < 1.0e-7) ratio = 1.0e-7;
    return span + (woofer - span) * pow(ratio, 10.0 - alpha);
}

/* The span a point receives from its three errors: the least-error span (0
 * when none qualifies), then the bass shift. */
static double point_span(const double err[3], const double spans[3], double alpha)
{
    double e;
    const int k = least_error(err, &e);
    const double chosen = (k < 0) ? 0.0 : spans[k];
    return bass_shift(chosen, e, err[2], spans[2], alpha);
}

/* Value of the variable-span fit at one point: the span is clipped to
 * [tweeter, woofer]; below the midrange span the midrange and tweeter fits
 * are mixed, otherwise the midrange and woofer fits, with the outer fit's
 * weight growing linearly from 0 at the midrange span to 1 at the outer
 * span. */
static double mix_fits(double span, const double spans[3], double f_tw, double f_mid, double f_wo)
{
    if (span <= spans[0]) span = spans[0];
    if (span >= spans[2]) span = spans[2];
    const int low = span - spans[1] < 0.0;
    const double outer_span = low ? spans[0] : spans[2];
    const double outer_fit = low ? f_tw : f_wo;
    const double g = (span - spans[1]) / (outer_span - spans[1]);
    return (1.0 - g) * f_mid + g * outer_fit;
}

/* ------------------------------------------------------------------ SS driver */

/* Super Smoother of one trial (Sec. 2.2, Friedman's variable-span smoother)
 * on sorted (x, y, w); spans = {tweeter, midrange, woofer}; iper as in
 * make_frame.  The stages:
 *   fits     for each span, the primary smooth of y with its leave-one-out
 *            residuals;
 *   errors   each span's residuals smoothed at the midrange span;
 *   spans    per point, point_span of the three errors;
 *   mixing   the per-point spans smoothed at the midrange span, then
 *            mix_fits of the three primary fits;
 *   result   the mixed curve smoothed at the tweeter span.
 * fixed_span > 0 replaces all of it by one smooth at that span. */
void ora_supsmu(int n, const double *x, const double *y, const double *w, int iper,
                const double *spans, double alpha, double fixed_span, double *smo)
{
    if (flat_phases(n, x, y, w, smo)) return;
    const ora_frame F = make_frame(n, x, w, iper);
    double *work = (double *)malloc((size_t)n * 9 * sizeof(double));
    double *scratch = work + 8 * (size_t)n;
    if (fixed_span > 0.0) {
        frame_smooth(&F, y, fixed_span, 1, smo, scratch, NULL);
        free(work);
        return;
    }
    /* candidate k: its primary fit and its smoothed CV error, point-major */
    struct {
        double *fit, *err;
    } cand[3];
    double *resid = work + 6 * (size_t)n, *span_pt = work + 7 * (size_t)n;
    for (int k = 0; k < 3; ++k) {
        cand[k].fit = work + (size_t)(2 * k) * n;
        cand[k].err = work + (size_t)(2 * k + 1) * n;
        frame_smooth(&F, y, spans[k], 1, cand[k].fit, resid, NULL);
        frame_smooth(&F, resid, spans[1], 0, cand[k].err, scratch, NULL);
    }
    for (int j = 0; j < n; ++j) {
        const double err[3] = {cand[0].err[j], cand[1].err[j], cand[2].err[j]};
        span_pt[j] = point_span(err, spans, alpha);
    }
    double *span_sm = resid; /* residuals no longer needed */
    frame_smooth(&F, span_pt, spans[1], 0, span_sm, scratch, NULL);
    double *mixed = span_pt;
    for (int j = 0; j < n; ++j)
        mixed[j] = mix_fits(span_sm[j], spans, cand[0].fit[j], cand[1].fit[j], cand[2].fit[j]);
    frame_smooth(&F, mixed, spans[0], 0, smo, scratch, NULL);
    free(work);
}

/* ------------------------------------------------------------------ SSSP (Sec. 3) */

/* Weighted residual sum of a fit. */
static double rss_of(int n, const double *y, const double *w, const double *fit)
{
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += w[j] * (y[j] - fit[j]) * (y[j] - fit[j]);
    return acc;
}

/* Trace of a smoother: sum of w_j h_j. */
static double trace_of(int n, const double *w, const double *lev)
{
    double acc = 0.0;
    for (int j = 0; j < n; ++j) acc += w[j] * lev[j];
    return acc;
}

/* One generalized-validation pass over K candidate spans.  Outputs per span
 * the weighted residual sum RSS_k (smooth after tie averaging) and the trace
 * TR_k = sum_j w_j h_j of the smoother; returns chi^2 = RSS of the first span
 * that minimises GCV_k = RSS_k/(1 - TR_k/n)^2 (GCV = +inf when TR_k >= n).
 * fixed_span > 0 replaces the candidates by that single span.  Flat phases
 * give the constant-mean fit of Sec. 2.2. */
double ora_sssp(int n, const double *x, const double *y, const double *w, int iper,
                const double *spans, int nspans, double fixed_span,
                double *rss_out, double *tr_out, int *kbest_out)
{
    double *fit = (double *)malloc((size_t)n * 3 * sizeof(double));
    double *r = fit + n, *lev = fit + 2 * n;
    double chi2;
    if (flat_phases(n, x, y, w, fit)) {
        chi2 = rss_of(n, y, w, fit);
        if (kbest_out) *kbest_out = -1;
        free(fit);
        return chi2;
    }
    const ora_frame F = make_frame(n, x, w, iper);
    const int K = (fixed_span > 0.0) ? 1 : nspans;
    double best = INFINITY;
    int kbest = 0;
    chi2 = NAN;
    for (int k = 0; k < K; ++k) {
        frame_smooth(&F, y, (fixed_span > 0.0) ? fixed_span : spans[k], 1, fit, r, lev);
        const double rss = rss_of(n, y, w, fit), tr = trace_of(n, w, lev);
        double gcv = INFINITY;
        if (tr < (double)n) {
            const double den = 1.0 - tr / (double)n;
            gcv = rss / (den * den);
        }
        if (rss_out) rss_out[k] = rss;
        if (tr_out) tr_out[k] = tr;
        if (k == 0 || gcv < best) {
            best = gcv;
            kbest = k;
            chi2 = rss;
        }
    }
    if (kbest_out) *kbest_out = kbest;
    free(fit);
    return chi2;
}

/* Second reading of the Sec. 3 variant (see the header): the three primary
 * fits and their traces from one pass; per point the error of span k is the
 * un-smoothed generalized-validation residual |y - s_k|/(1 - TR_k/n) (+inf
 * when TR_k >= n); point_span and mix_fits as in the Super Smoother, and
 * chi^2 of the mixed fit (no error, span or final smooth).  A fixed span is
 * the fixed-span smooth. */
double ora_sssp2(int n, const double *x, const double *y, const double *w, int iper,
                 const double *spans, double alpha, double fixed_span)
{
    double *work = (double *)malloc((size_t)n * 6 * sizeof(double));
    double *fit[3] = {work, work + n, work + 2 * n};
    double *r = work + 3 * n, *lev = work + 4 * n, *mixed = work + 5 * n;
    double chi2;
    if (flat_phases(n, x, y, w, mixed)) {
        chi2 = rss_of(n, y, w, mixed);
        free(work);
        return chi2;
    }
    const ora_frame F = make_frame(n, x, w, iper);
    if (fixed_span > 0.0) {
        frame_smooth(&F, y, fixed_span, 1, mixed, r, lev);
        chi2 = rss_of(n, y, w, mixed);
        free(work);
        return chi2;
    }
    double gv_den[3];
    int usable[3];
    for (int k = 0; k < 3; ++k) {
        frame_smooth(&F, y, spans[k], 1, fit[k], r, lev);
        const double tr = trace_of(n, w, lev);
        usable[k] = tr < (double)n;
        gv_den[k] = 1.0 - tr / (double)n;
    }
    for (int j = 0; j < n; ++j) {
        double err[3];
        for (int k = 0; k < 3; ++k)
            err[k] = usable[k] ? fabs(y[j] - fit[k][j]) / gv_den[k] : INFINITY;
        mixed[j] = mix_fits(point_span(err, spans, alpha), spans, fit[0][j], fit[1][j], fit[2][j]);
    }
    chi2 = rss_of(n, y, w, mixed);
    free(work);
    return chi2;
}

/* Phase dispersion score of one trial: phase = (tt mod p)/p, bin =
 * floor(phase B) (clamped to B - 1), score = sum_b (sum w (y - ybar))^2 /
 * (sum w) over the non-empty bins, divided by chi0; ybar is the weighted
 * mean.  The bins need no sort. */
double ora_pdm(int n, const double *tt, const double *y, const double *w, double ybar,
               double chi0, double f, int B)
{
    double *ph = (double *)malloc((size_t)n * sizeof(double));
    double *acc = (double *)calloc((size_t)(2 * B), sizeof(double));
    ora_fold(n, tt, f, ph);
    for (int i = 0; i < n; ++i) {
        int b = (int)floor(ph[i] * (double)B);
        if (b > B - 1) b = B - 1;
        if (b < 0) b = 0;
        acc[b] += w[i];
        acc[B + b] += w[i] * (y[i] - ybar);
    }
    double e = 0.0;
    for (int b = 0; b < B; ++b)
        if (acc[b] > 0.0) e += acc[B + b] * acc[B + b] / acc[b];
    free(acc);
    free(ph);
    return e / chi0;
}

/* ------------------------------------------------------------------ one trial */

/* One (object, frequency) trial: fold, stable sort, smoother, chi^2, P.
 * tt, y, w come from ora_prep (original order).  iper as in ora_supsmu. */
double ora_trial(int method, int n, const double *tt, const double *y, const double *w,
                 double chi0, double f, int iper, const double *spans, double alpha,
                 double fixed_span)
{
    double *ph = (double *)malloc((size_t)n * 5 * sizeof(double));
    double *xs = ph + n, *ys = ph + 2 * n, *ws = ph + 3 * n, *smo = ph + 4 * n;
    int64_t *perm = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    ora_fold(n, tt, f, ph);
    ora_argsort(n, ph, perm);
    for (int j = 0; j < n; ++j) {
        xs[j] = ph[perm[j]];
        ys[j] = y[perm[j]];
        ws[j] = w[perm[j]];
    }
    double chi2;
    if (method == ORA_METHOD_SS) {
        ora_supsmu(n, xs, ys, ws, iper, spans, alpha, fixed_span, smo);
        chi2 = 0.0;
        for (int j = 0; j < n; ++j) chi2 += ws[j] * (ys[j] - smo[j]) * (ys[j] - smo[j]);
    } else if (method == ORA_METHOD_SSSP) {
        chi2 = ora_sssp(n, xs, ys, ws, iper, spans, 3, fixed_span, NULL, NULL, NULL);
    } else {
        chi2 = ora_sssp2(n, xs, ys, ws, iper, spans, alpha, fixed_span);
    }
    free(perm);
    free(ph);
    return 1.0 - chi2 / chi0;
}

/* ------------------------------------------------------------------ catalog */

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Periodogram of a catalog in CSR form (offsets[n_obj+1], values per object
 * contiguous).  ks selects frequency indices (NULL = all n_freq); the output
 * is pgram[o*nk + i] for the i-th selected index.  Objects with a non-OK
 * status get NaN rows.  Parallel over (object, frequency) pairs. */
void ora_periodogram(int method, int64_t n_obj, const int64_t *offsets, const double *t,
                     const double *y, const double *e, double fmin, double fmax,
                     int64_t n_freq, const int64_t *ks, int64_t nk, const double *spans,
                     double alpha, double fixed_span, double *pgram, int32_t *status)
{
    if (!ks) nk = n_freq;
    double *tt = (double *)malloc((size_t)offsets[n_obj] * sizeof(double) + 8);
    double *w = (double *)malloc((size_t)offsets[n_obj] * sizeof(double) + 8);
    double *chi0 = (double *)malloc((size_t)n_obj * sizeof(double) + 8);
    for (int64_t o = 0; o < n_obj; ++o) {
        int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
        status[o] = ora_prep(n, t + a, y + a, e + a, tt + a, w + a, NULL, chi0 + o);
    }
    int64_t total = n_obj * nk;
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t it = 0; it < total; ++it) {
        int64_t o = it / nk, i = it % nk;
        if (status[o] != ORA_OK) {
            pgram[it] = NAN;
            continue;
        }
        int64_t k = ks ? ks[i] : i;
        int64_t a = offsets[o], n = offsets[o + 1] - offsets[o];
        double f = ora_freq(fmin, fmax, n_freq, k);
        pgram[it] = ora_trial(method, (int)n, tt + a, y + a, w + a, chi0[o], f, 2, spans,
                              alpha, fixed_span);
    }
    free(tt);
    free(w);
    free(chi0);
}

/* findPeriod: index of the largest P (lowest index among equal maxima, NaN
 * skipped); -1 when every value is NaN. */
int64_t ora_best(int64_t nk, const double *p)
{
    int64_t best = -1;
    for (int64_t i = 0; i < nk; ++i) {
        if (isnan(p[i])) continue;
        if (best < 0 || p[i] > p[best]) best = i;
    }
    return best;
}
