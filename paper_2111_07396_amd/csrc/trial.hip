// Fused per-trial kernel: fold -> LDS bucket sort -> Super Smoother (Listing
// 1) or the single-pass GCV variant (Sec. 3) -> chi^2 -> P -> tile argmax.
//
// One wavefront owns one (object, frequency tile) work item and runs its
// trials one after another, PPL consecutive sorted points per lane.
// Arithmetic follows the policy P (numeric.hpp): FP64, or FP32 with
// compensated float-pair sums.
//
// Every running-line smooth is a pair of window sums (of w v and w x v)
// combined with the window's geometry (numeric.hpp, Geo), and the geometry
// depends only on the sorted phases and the span.  A trial therefore
//   phase A: builds prefix sums of w, w x, w x^2 and of w y, w x y; computes
//            the geometry of the three spans once, and with it the three
//            cross-validated smooths of y (Listing 1's primaries);
//   phase B: smooths the three |CV residuals|, the chosen spans and the blend
//            with the stored midrange / tweeter geometry, one prefix pair each.
// A window that wraps around the phase cycle is read from the periodic
// extension of the prefix sums (x shifted by +-1 on the far side).
// Prefix arrays are stored with one pad slot per lane chunk when PPL is even,
// so that the 64 lanes' reads at a common offset fall in distinct LDS banks.
#include "numeric.hpp"
#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

constexpr int kWavesPerBlock = 2;

__host__ __device__ constexpr int align16(int b) { return (b + 15) / 16 * 16; }

template <int PPL>
struct Lay {
    static constexpr int NP = kWave * PPL;
    static constexpr bool SKEW = (PPL % 2) == 0;
    static constexpr int NS = NP + (SKEW ? kWave : 0) + 1;  // slots of a prefix array
    static constexpr int A8 = align16(NS * 8);
    // phase A: x-moments (X0..X2) and y (Y0, Y1).  Phase B: X0, X1 hold the
    // prefix pair of the smoothed quantity, X2 and Y0, Y1 are scratch.
    static constexpr int X0 = 0, X1 = A8, X2 = 2 * A8, Y0 = 3 * A8, Y1 = 4 * A8;
    static constexpr int SMOOTH_END = 5 * A8;
    // sort scratch (aliases the prefix arrays; dead once the sort is done)
    static constexpr int CNT = 0;
    static constexpr int TMP = align16((NP + 1) * 4);
    static constexpr int SY = TMP + NP * 8;
    static constexpr int SW = SY + NP * 8;
    static constexpr int SORT_END = SW + NP * 8;
    // sorted keys live for the whole trial
    static constexpr int SK = align16(SMOOTH_END > SORT_END ? SMOOTH_END : SORT_END);
    static constexpr int BYTES = SK + NP * 8;
};

template <int PPL>
__device__ __forceinline__ int sidx(int j) {
    return Lay<PPL>::SKEW ? j + j / PPL : j;
}

template <class P>
struct Trial {
    using S = typename P::S;
    S *X0, *X1, *X2, *Y0, *Y1;
    const uint64_t *SK;
    int n, lane;
    double vsmlsq;
    bool ties;
};

// Half-window of a span: b = max(2, floor(0.5*span*n + 0.5)), clamped so
// that 2b+1 <= n.
__device__ __forceinline__ int halfwidth(int n, double span) {
    int b = (int)halfwidth_real(span, n);
    if (b < 2) b = 2;
    if (2 * b + 1 > n) b = (n - 1) / 2;
    return b;
}

// tmp^e for the bass enhancement, 1e-7 <= tmp <= 1.  Whole exponents (the
// paper's alpha = 9 gives e = 1) by repeated products; otherwise through the
// FP32 exp2/log2 units (relative error ~1e-7 of the span increment).
template <class P>
__device__ __forceinline__ typename P::R bass_pow(typename P::R tmp, typename P::R e) {
    using R = typename P::R;
    if (e == __builtin_floor((double)e) && e >= R(0) && e <= R(10)) {
        R r = R(1);
        for (int i = 0; i < (int)e; ++i) r *= tmp;
        return r;
    }
    return P::exp2_log2_pow(tmp, e);
}

// Writes the exclusive prefix sums Pf[j] = sum_{i<j} v_i of M quantities
// (Pf[0] = 0, Pf[j+1] after point j); padding points contribute 0.
template <class P, int PPL, int M>
__device__ __forceinline__ void build_prefix(typename P::S *const (&Pf)[M],
                                             const typename P::S (&v)[M][PPL], int lane) {
    using S = typename P::S;
    S loc[M][PPL];
    S tot[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
        S acc = v[m][0];
        loc[m][0] = acc;
#pragma unroll
        for (int p = 1; p < PPL; ++p) {
            acc = P::add(acc, v[m][p]);
            loc[m][p] = acc;
        }
        tot[m] = acc;
    }
    S excl[M];
#pragma unroll
    for (int m = 0; m < M; ++m) excl[m] = P::sub(P::scan(tot[m]), tot[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) {
#pragma unroll
        for (int p = 0; p < PPL; ++p) Pf[m][sidx<PPL>(lane * PPL + p + 1)] = P::add(excl[m], loc[m][p]);
        if (lane == 0) Pf[m][0] = P::zero();
    }
}

// Window [j-b, j+b] of point j from prefix sums P (P[i] = sum over points
// 0..i-1).  With lo = j-b and hi = j+b+1 the window is the difference of the
// prefix at B = hi (hi - n if hi > n) and at A = lo (lo + n if lo < 0), plus
// the totals T once if it wraps (c = 1).  The wrapped part carries its phase
// shifted by d = +1 (right end, points 0 .. hi-n-1: prefix B) or d = -1 (left
// end, points n+lo .. n-1: totals minus prefix A); Q is its weighted sum of a
// quantity, so shifting x by d adds d Q_w to the sum of w x, 2 d Q_x + Q_w to
// the sum of w x^2 and d Q_v to the sum of w x v.
struct WinIdx {
    int a, b;
    float c, d, sr, sl;  // 0/1 flags and d = sr - sl
};
template <int PPL>
__device__ __forceinline__ WinIdx win_idx(int j, int b, int n) {
    const int lo = j - b, hi = j + b + 1;
    const bool left = lo < 0, right = hi > n;
    WinIdx w;
    w.a = sidx<PPL>(left ? lo + n : lo);
    w.b = sidx<PPL>(right ? hi - n : hi);
    w.sl = left ? 1.0f : 0.0f;
    w.sr = right ? 1.0f : 0.0f;
    w.c = w.sl + w.sr;
    w.d = w.sr - w.sl;
    return w;
}

template <class P>
struct Sum3 {
    typename P::S w, x, xx;
};
template <class P>
struct Sum2 {
    typename P::S v, xv;
};

template <class P, int PPL>
__device__ __forceinline__ Sum3<P> window3(const Trial<P> &T, const Sum3<P> &tot, const WinIdx &ix) {
    using R = typename P::R;
    const R c = (R)ix.c, d = (R)ix.d, sr = (R)ix.sr, sl = (R)ix.sl;
    const auto aw = T.X0[ix.a], ax = T.X1[ix.a], axx = T.X2[ix.a];
    const auto bw = T.X0[ix.b], bx = T.X1[ix.b], bxx = T.X2[ix.b];
    const auto qw = P::add(P::scale(bw, sr), P::scale(P::sub(tot.w, aw), sl));
    const auto qx = P::add(P::scale(bx, sr), P::scale(P::sub(tot.x, ax), sl));
    Sum3<P> s;
    s.w = P::add(P::sub(bw, aw), P::scale(tot.w, c));
    s.x = P::add(P::add(P::sub(bx, ax), P::scale(tot.x, c)), P::scale(qw, d));
    s.xx = P::add(P::add(P::sub(bxx, axx), P::scale(tot.xx, c)),
                  P::add(P::scale(P::twice(qx), d), P::scale(qw, c)));
    return s;
}

template <class P, int PPL>
__device__ __forceinline__ Sum2<P> window2(const typename P::S *PV, const typename P::S *PXV,
                                           const Sum2<P> &tot, const WinIdx &ix) {
    using R = typename P::R;
    const R c = (R)ix.c, d = (R)ix.d, sr = (R)ix.sr, sl = (R)ix.sl;
    const auto av = PV[ix.a], axv = PXV[ix.a];
    const auto bv = PV[ix.b], bxv = PXV[ix.b];
    const auto qv = P::add(P::scale(bv, sr), P::scale(P::sub(tot.v, av), sl));
    Sum2<P> s;
    s.v = P::add(P::sub(bv, av), P::scale(tot.v, c));
    s.xv = P::add(P::add(P::sub(bxv, axv), P::scale(tot.xv, c)), P::scale(qv, d));
    return s;
}

template <class P, int PPL>
__device__ __forceinline__ typename P::Geo geometry(const Trial<P> &T, const Sum3<P> &tot,
                                                    const WinIdx &ix, typename P::S xj,
                                                    typename P::R &h) {
    const Sum3<P> s = window3<P, PPL>(T, tot, ix);
    return P::geo(s.w, s.x, s.xx, xj, T.vsmlsq, h);
}

template <class P, int PPL>
__device__ __forceinline__ typename P::R window_fit(const typename P::S *PV,
                                                    const typename P::S *PXV,
                                                    const Sum2<P> &tot,
                                                    const typename P::Geo &g, const WinIdx &ix) {
    const Sum2<P> s = window2<P, PPL>(PV, PXV, tot, ix);
    return P::eval(g, s.v, s.xv);
}

// Prefix pair of w v and w x v into (PV, PXV); returns the totals.
template <class P, int PPL>
__device__ __forceinline__ Sum2<P> prefix_pair(typename P::S *PV, typename P::S *PXV, int n,
                                               int lane, const typename P::R (&w)[PPL],
                                               const typename P::S (&wx)[PPL],
                                               const typename P::R (&v)[PPL]) {
    using S = typename P::S;
    S q[2][PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        q[0][p] = P::prod(w[p], v[p]);
        q[1][p] = P::mulr(wx[p], v[p]);
    }
    S *const Pf[2] = {PV, PXV};
    wave_lds_sync();
    build_prefix<P, PPL, 2>(Pf, q, lane);
    wave_lds_sync();
    const int r = sidx<PPL>(n);
    return Sum2<P>{PV[r], PXV[r]};
}

// ---- rare paths, kept out of line: they work on LDS only, so no register
// arrays cross the call.

// out[j] (j in [j0, j1)) = weighted mean of s over the run of equal phase
// holding j, or s[j] when the phase of j is unique.
template <class R>
__device__ __noinline__ void tie_means(const R *s, const R *w, R *out, const uint64_t *SK, int n,
                                       int j0, int j1) {
    for (int j = j0; j < j1; ++j) {
        const uint64_t xj = SK[j] >> 16;
        int a = j, b = j;
        while (a > 0 && (SK[a - 1] >> 16) == xj) --a;
        while (b + 1 < n && (SK[b + 1] >> 16) == xj) ++b;
        if (a == b) {
            out[j] = s[j];
            continue;
        }
        double sws = 0.0, sw = 0.0;
        for (int i = a; i <= b; ++i) {
            sws += (double)w[i] * (double)s[i];
            sw += (double)w[i];
        }
        out[j] = sw > 0.0 ? (R)(sws / sw) : R(0);
    }
}

// out[j] = r[j] where r[j] >= 0, else the nearest earlier non-negative r
// (0 if none): the CV residual of a point with 1 - w h <= 0.
template <class R>
__device__ __noinline__ void fallback_fill(const R *r, R *out, int j0, int j1) {
    for (int j = j0; j < j1; ++j) {
        if (r[j] >= R(0)) {
            out[j] = r[j];
            continue;
        }
        int i = j - 1;
        while (i >= 0 && r[i] < R(0)) --i;
        out[j] = i >= 0 ? r[i] : R(0);
    }
}

// Replaces s over every run of equal phase by the run's weighted mean (uses
// X0..X2 as scratch: they must be dead).
template <class P, int PPL>
__device__ void tie_average(const Trial<P> &T, const typename P::R (&w)[PPL],
                            typename P::R (&s)[PPL]) {
    using R = typename P::R;
    R *S1 = (R *)T.X0, *S2 = (R *)T.X1, *S3 = (R *)T.X2;
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = T.lane * PPL + p;
        if (j < T.n) {
            S1[j] = s[p];
            S2[j] = w[p];
        }
    }
    wave_lds_sync();
    const int j0 = min(T.lane * PPL, T.n), j1 = min(T.lane * PPL + PPL, T.n);
    tie_means<R>(S1, S2, S3, T.SK, T.n, j0, j1);
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = T.lane * PPL + p;
        if (j < T.n) s[p] = S3[j];
    }
    wave_lds_sync();
}

// Leave-one-out residual |v - s|/(1 - w h); -1 marks 1 - w h <= 0.
template <class P>
__device__ __forceinline__ typename P::R cv_resid(typename P::R v, typename P::R s,
                                                  typename P::R w, typename P::R h) {
    using R = typename P::R;
    const R d = R(1) - w * h;
    return d > R(0) ? P::fabs_(v - s) * P::rcp(d) : R(-1);
}

// Where 1 - w h <= 0 the residual repeats the previous point's (0 at j = 0).
// Uses X1, X2 as scratch.
template <class P, int PPL>
__device__ void cv_fallback(const Trial<P> &T, typename P::R (&r)[PPL]) {
    using R = typename P::R;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < PPL; ++p) bad |= (T.lane * PPL + p < T.n) && r[p] < R(0);
    if (wave_ballot(bad) == 0) return;
    R *S1 = (R *)T.X1, *S2 = (R *)T.X2;
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = T.lane * PPL + p;
        if (j < T.n) S1[j] = r[p];
    }
    wave_lds_sync();
    fallback_fill<R>(S1, S2, min(T.lane * PPL, T.n), min(T.lane * PPL + PPL, T.n));
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = T.lane * PPL + p;
        if (j < T.n) r[p] = S2[j];
    }
    wave_lds_sync();
}

// Weighted residual sum, accumulated per lane in the policy's sum type and
// reduced across the wave in FP64.
template <class P, int PPL>
__device__ __forceinline__ double wave_chi2(const Trial<P> &T, const typename P::R (&w)[PPL],
                                            const typename P::R (&y)[PPL],
                                            const typename P::R (&smo)[PPL]) {
    using R = typename P::R;
    auto acc = P::zero();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const R d = T.lane * PPL + p < T.n ? y[p] - smo[p] : R(0);
        acc = P::add(acc, P::prod(w[p] * d, d));
    }
    return wave_sum(P::dbl(acc));
}

// Smooth of v with a stored geometry (phase B): prefix pair in X0/X1, ties.
template <class P, int PPL>
__device__ __forceinline__ void smooth_with(const Trial<P> &T, int b,
                                           const typename P::Geo (&g)[PPL],
                                           const typename P::R (&w)[PPL],
                                           const typename P::S (&wx)[PPL],
                                           const typename P::R (&v)[PPL],
                                           typename P::R (&s)[PPL]) {
    const Sum2<P> tot = prefix_pair<P, PPL>(T.X0, T.X1, T.n, T.lane, w, wx, v);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const WinIdx ix = win_idx<PPL>(min(T.lane * PPL + p, T.n - 1), b, T.n);
        s[p] = window_fit<P, PPL>(T.X0, T.X1, tot, g[p], ix);
    }
    if (T.ties) tie_average<P, PPL>(T, w, s);
}

// Listing 1 on the sorted trial; returns chi^2.
template <class P, int PPL>
__device__ double supersmoother(Trial<P> &T, const TrialLaunch &L, const typename P::S (&x)[PPL],
                                const typename P::R (&w)[PPL], const typename P::S (&wx)[PPL],
                                const typename P::R (&y)[PPL], const Sum3<P> &xt,
                                const Sum2<P> &yt) {
    using R = typename P::R;
    using Geo = typename P::Geo;
    const int n = T.n, lane = T.lane;
    if (L.fixed_span > 0.0) {  // Listing 1: one smooth at the fixed span
        const int b = halfwidth(n, L.fixed_span);
        R smo[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const WinIdx ix = win_idx<PPL>(min(lane * PPL + p, n - 1), b, n);
            R h;
            const Geo g = geometry<P, PPL>(T, xt, ix, x[p], h);
            smo[p] = window_fit<P, PPL>(T.Y0, T.Y1, yt, g, ix);
        }
        if (T.ties) tie_average<P, PPL>(T, w, smo);
        return wave_chi2<P, PPL>(T, w, y, smo);
    }
    const int b0 = halfwidth(n, L.span[0]), b1 = halfwidth(n, L.span[1]),
              b2 = halfwidth(n, L.span[2]);
    const R sp0 = (R)L.span[0], sp1 = (R)L.span[1], sp2 = (R)L.span[2];

    // ---- phase A: geometry of the three spans and the cross-validated
    // smooths of y (tweeter, midrange, woofer) with their |CV residuals|
    Geo g0[PPL], g1[PPL];
    R s0[PPL], s1[PPL], s2[PPL], r0[PPL], r1[PPL], r2[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = min(lane * PPL + p, n - 1);
        R h;
        WinIdx ix = win_idx<PPL>(j, b0, n);
        g0[p] = geometry<P, PPL>(T, xt, ix, x[p], h);
        s0[p] = window_fit<P, PPL>(T.Y0, T.Y1, yt, g0[p], ix);
        r0[p] = cv_resid<P>(y[p], s0[p], w[p], h);
        ix = win_idx<PPL>(j, b1, n);
        g1[p] = geometry<P, PPL>(T, xt, ix, x[p], h);
        s1[p] = window_fit<P, PPL>(T.Y0, T.Y1, yt, g1[p], ix);
        r1[p] = cv_resid<P>(y[p], s1[p], w[p], h);
        ix = win_idx<PPL>(j, b2, n);
        const Geo g2 = geometry<P, PPL>(T, xt, ix, x[p], h);
        s2[p] = window_fit<P, PPL>(T.Y0, T.Y1, yt, g2, ix);
        r2[p] = cv_resid<P>(y[p], s2[p], w[p], h);
    }
    // ---- phase B (the phase-A prefix arrays are free): fallbacks and ties
    // of the primaries
    cv_fallback<P, PPL>(T, r0);
    cv_fallback<P, PPL>(T, r1);
    cv_fallback<P, PPL>(T, r2);
    if (T.ties) {
        tie_average<P, PPL>(T, w, s0);
        tie_average<P, PPL>(T, w, s1);
        tie_average<P, PPL>(T, w, s2);
    }
    // midrange smooths of the residuals; per-point span choice, the lowest
    // span winning ties (Listing 1 scans the spans upward with a strict <,
    // starting from 1e20; the span stays 0 if no residual is below that)
    R resmin[PPL], sel[PPL], rt[PPL];
    smooth_with<P, PPL>(T, b1, g1, w, wx, r0, rt);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const bool lt = rt[p] < R(1.0e20);
        resmin[p] = lt ? rt[p] : R(1.0e20);
        sel[p] = lt ? sp0 : R(0);
    }
    smooth_with<P, PPL>(T, b1, g1, w, wx, r1, rt);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const bool lt = rt[p] < resmin[p];
        resmin[p] = lt ? rt[p] : resmin[p];
        sel[p] = lt ? sp1 : sel[p];
    }
    smooth_with<P, PPL>(T, b1, g1, w, wx, r2, rt);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const bool lt = rt[p] < resmin[p];
        resmin[p] = lt ? rt[p] : resmin[p];
        sel[p] = lt ? sp2 : sel[p];
    }
    // bass enhancement against the woofer's smoothed residual
    const double alpha = L.alpha;
    if (alpha > 0.0 && alpha <= 10.0) {
        const R ex = (R)(10.0 - alpha);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            if (resmin[p] < rt[p] && resmin[p] > R(0)) {
                R tmp = resmin[p] / rt[p];
                if (tmp < R(1.0e-7)) tmp = R(1.0e-7);
                sel[p] += (sp2 - sel[p]) * bass_pow<P>(tmp, ex);
            }
        }
    }
    // midrange smooth of the chosen spans, clip, blend
    smooth_with<P, PPL>(T, b1, g1, w, wx, sel, rt);
    const R ilo = R(1) / (sp0 - sp1), ihi = R(1) / (sp2 - sp1);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        R sj = rt[p];
        if (sj <= sp0) sj = sp0;
        if (sj >= sp2) sj = sp2;
        const R f = sj - sp1;
        const bool below = f < R(0);
        const R fr = below ? f * ilo : f * ihi;
        rt[p] = (R(1) - fr) * s1[p] + fr * (below ? s0[p] : s2[p]);
    }
    // tweeter smooth of the blend
    R smo[PPL];
    smooth_with<P, PPL>(T, b0, g0, w, wx, rt, smo);
    return wave_chi2<P, PPL>(T, w, y, smo);
}

// Sec. 3 single pass: one prefix of y serves every candidate span.
template <class P, int PPL>
__device__ double single_pass(Trial<P> &T, const TrialLaunch &L, const typename P::S (&x)[PPL],
                              const typename P::R (&w)[PPL], const typename P::R (&y)[PPL],
                              const Sum3<P> &xt, const Sum2<P> &yt) {
    using R = typename P::R;
    using Geo = typename P::Geo;
    const int n = T.n, lane = T.lane;
    const int K = L.fixed_span > 0.0 ? 1 : 3;
    int b[3];
    for (int k = 0; k < 3; ++k) b[k] = halfwidth(n, K == 1 ? L.fixed_span : L.span[k]);
    R s[3][PPL];
    typename P::S tr[3] = {P::zero(), P::zero(), P::zero()};
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = min(lane * PPL + p, n - 1);
        const bool ok = lane * PPL + p < n;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            s[k][p] = R(0);
            if (k < K) {
                const WinIdx ix = win_idx<PPL>(j, b[k], n);
                R h;
                const Geo g = geometry<P, PPL>(T, xt, ix, x[p], h);
                s[k][p] = window_fit<P, PPL>(T.Y0, T.Y1, yt, g, ix);
                tr[k] = P::add(tr[k], P::prod(ok ? w[p] : R(0), h));
            }
        }
    }
    if (T.ties) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < K) tie_average<P, PPL>(T, w, s[k]);
    }
    double best = 0.0, chi2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= K) break;
        auto rss = P::zero();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const R d = lane * PPL + p < n ? y[p] - s[k][p] : R(0);
            rss = P::add(rss, P::prod(w[p] * d, d));
        }
        const double rss_d = wave_sum(P::dbl(rss));
        const double tr_d = wave_sum(P::dbl(tr[k]));
        double gcv = __builtin_inf();
        if (tr_d < (double)n) {
            const double den = 1.0 - tr_d / (double)n;
            gcv = rss_d / (den * den);
        }
        if (k == 0 || gcv < best) {
            best = gcv;
            chi2 = rss_d;
        }
    }
    return chi2;
}

// Object data of the work item, original (time) order; re-read from the
// caches at every trial instead of being held in registers.
template <class P>
struct ObjData {
    const double *tt;
    const typename P::R *y, *w;
};

template <class P, int PPL, int METHOD>
__device__ double run_trial(unsigned char *lds, int lane, int n, const TrialLaunch &L,
                            const ObjData<P> &od, double f, double chi0) {
    using R = typename P::R;
    using S = typename P::S;
    using Y = Lay<PPL>;
    constexpr int NP = Y::NP;
    // ---- fold (FP64): phase = frac(tt*f), as a 48-bit fixed-point key with
    // the point index in the low 16 bits (stable order on equal phases)
    uint64_t key[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = lane * PPL + p;
        const double u = od.tt[min(j, n - 1)] * f;
        const double ph = u - floor(u);
        const uint64_t ph48 = (uint64_t)(ph * 0x1p48);
        key[p] = j < n ? ((ph48 << 16) | (uint64_t)j) : ~0ull;
    }
    // ---- bucket sort in LDS: NP buckets on the top phase bits, counts by LDS
    // atomics, a wave scan for the bucket starts, then the exact rank inside a
    // bucket by comparing against its (few) members.
    uint32_t *cnt = (uint32_t *)(lds + Y::CNT);
    uint64_t *tmp = (uint64_t *)(lds + Y::TMP);
    R *sy = (R *)(lds + Y::SY);
    R *sw = (R *)(lds + Y::SW);
    uint64_t *SK = (uint64_t *)(lds + Y::SK);
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) cnt[lane * PPL + p] = 0u;
    wave_lds_sync();
    int bkt[PPL];
    uint32_t slot[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = lane * PPL + p;
        bkt[p] = (int)(((key[p] >> 32) * (uint64_t)NP) >> 32);
        slot[p] = 0u;
        if (j < n) slot[p] = atomicAdd(&cnt[bkt[p]], 1u);
    }
    wave_lds_sync();
    {
        uint32_t c[PPL], tot = 0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            c[p] = cnt[lane * PPL + p];
            tot += c[p];
        }
        const uint32_t incl = wave_incl_sum_u32(tot);
        uint32_t run = incl - tot;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            cnt[lane * PPL + p] = run;
            run += c[p];
        }
        if (lane == kWave - 1) cnt[NP] = incl;
    }
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = lane * PPL + p;
        if (j < n) tmp[cnt[bkt[p]] + slot[p]] = key[p];
    }
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = lane * PPL + p;
        if (j < n) {
            const uint32_t s = cnt[bkt[p]], e = cnt[bkt[p] + 1];
            uint32_t rank = 0;
            for (uint32_t i = s; i < e; ++i) rank += tmp[i] < key[p] ? 1u : 0u;
            const uint32_t pos = s + rank;
            SK[pos] = key[p];
            sy[pos] = od.y[j];
            sw[pos] = od.w[j];
        }
    }
    wave_lds_sync();
    S x[PPL], wx[PPL];
    R y[PPL], w[PPL];
    uint64_t klast = 0;
    bool tie = false;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = lane * PPL + p;
        const bool ok = j < n;
        const uint64_t k = ok ? SK[j] : ~0ull;
        y[p] = ok ? sy[j] : R(0);
        w[p] = ok ? sw[j] : R(0);
        x[p] = ok ? P::x_of_key(k) : P::zero();
        wx[p] = P::mulr(x[p], w[p]);
        if (j + 1 < n) tie |= (SK[j + 1] >> 16) == (k >> 16);
        (void)klast;
    }
    wave_lds_sync();

    Trial<P> T;
    T.X0 = (S *)(lds + Y::X0);
    T.X1 = (S *)(lds + Y::X1);
    T.X2 = (S *)(lds + Y::X2);
    T.Y0 = (S *)(lds + Y::Y0);
    T.Y1 = (S *)(lds + Y::Y1);
    T.SK = SK;
    T.n = n;
    T.lane = lane;
    T.ties = wave_ballot(tie) != 0;

    // ---- Listing 1: constant fit when the phases do not spread
    if ((SK[n - 1] >> 16) <= (SK[0] >> 16)) {
        double a = 0.0, sw_ = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            a += (double)w[p] * (double)y[p];
            sw_ += (double)w[p];
        }
        a = wave_sum(a);
        sw_ = wave_sum(sw_);
        const R m = (R)(sw_ > 0.0 ? a / sw_ : 0.0);
        R smo[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) smo[p] = m;
        return 1.0 - wave_chi2<P, PPL>(T, w, y, smo) / chi0;
    }
    {
        const int q = n / 4;
        const double scale = (double)(SK[3 * q - 1] >> 16) * 0x1p-48 -
                             (double)(SK[q - 1] >> 16) * 0x1p-48;
        T.vsmlsq = listing_vsmlsq(scale);
    }
    // ---- phase A prefix sums: x-moments and y, shared by all three spans
    Sum3<P> xt;
    Sum2<P> yt;
    {
        S q[5][PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            q[0][p] = P::from(w[p]);
            q[1][p] = wx[p];
            q[2][p] = P::mul(wx[p], x[p]);
            q[3][p] = P::prod(w[p], y[p]);
            q[4][p] = P::mulr(wx[p], y[p]);
        }
        S *const Pf[5] = {T.X0, T.X1, T.X2, T.Y0, T.Y1};
        build_prefix<P, PPL, 5>(Pf, q, lane);
        wave_lds_sync();
        const int r = sidx<PPL>(n);
        xt = Sum3<P>{T.X0[r], T.X1[r], T.X2[r]};
        yt = Sum2<P>{T.Y0[r], T.Y1[r]};
    }
    const double chi2 = (METHOD == 0) ? supersmoother<P, PPL>(T, L, x, w, wx, y, xt, yt)
                                      : single_pass<P, PPL>(T, L, x, w, y, xt, yt);
    return 1.0 - chi2 / chi0;
}

template <class P, int PPL, int METHOD>
__global__ __launch_bounds__(kWave *kWavesPerBlock) void trial_kernel(TrialLaunch L) {
    using R = typename P::R;
    extern __shared__ __align__(16) unsigned char smem[];
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wave;
    if (item >= L.n_items) return;
    unsigned char *lds = smem + wave * Lay<PPL>::BYTES;
    const int64_t ci = item / L.n_tiles;
    const int32_t tile = (int32_t)(item - ci * L.n_tiles);
    const int obj = L.objs[ci];
    const int64_t k0 = (int64_t)tile * L.tile_f;
    const int64_t k1 = (k0 + L.tile_f < L.n_freq) ? k0 + L.tile_f : L.n_freq;
    const int64_t part = (int64_t)obj * L.n_tiles + tile;
    const int64_t row = (int64_t)obj * L.n_freq;

    if (L.cat.status[obj] != 0) {
        for (int64_t k = k0 + lane; k < k1; k += kWave) {
            if (L.pgram64) L.pgram64[row + k] = __builtin_nan("");
            if (L.pgram32) L.pgram32[row + k] = __builtin_nanf("");
        }
        if (lane == 0 && L.part_p) {
            L.part_p[part] = __builtin_nan("");
            L.part_k[part] = -1;
        }
        return;
    }
    const int64_t base = L.cat.offsets[obj];
    const int n = (int)(L.cat.offsets[obj + 1] - base);
    ObjData<P> od;
    od.tt = L.cat.tt + base;
    od.y = (P::kIsF64 ? (const R *)L.cat.yc : (const R *)L.cat.yc32) + base;
    od.w = (P::kIsF64 ? (const R *)L.cat.w : (const R *)L.cat.w32) + base;
    const double chi0 = L.cat.chi0[obj];
    double best_p = 0.0;
    int32_t best_k = -1;
    for (int64_t k = k0; k < k1; ++k) {
        const double f = grid_freq(L.fmin, L.df, k);
        const double Pk = run_trial<P, PPL, METHOD>(lds, lane, n, L, od, f, chi0);
        if (lane == 0) {
            if (L.pgram64) L.pgram64[row + k] = Pk;
            if (L.pgram32) L.pgram32[row + k] = (float)Pk;
        }
        if (!__builtin_isnan(Pk) && (best_k < 0 || Pk > best_p)) {
            best_p = Pk;
            best_k = (int32_t)k;
        }
    }
    if (lane == 0 && L.part_p) {
        L.part_p[part] = best_k < 0 ? __builtin_nan("") : best_p;
        L.part_k[part] = best_k;
    }
}

template <class P, int PPL, int METHOD>
hipError_t launch_one(const TrialLaunch &L, hipStream_t s) {
    const size_t lds = (size_t)Lay<PPL>::BYTES * kWavesPerBlock;
    hipError_t e = hipFuncSetAttribute((const void *)trial_kernel<P, PPL, METHOD>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const int64_t blocks = (L.n_items + kWavesPerBlock - 1) / kWavesPerBlock;
    hipLaunchKernelGGL((trial_kernel<P, PPL, METHOD>), dim3((unsigned)blocks),
                       dim3(kWave * kWavesPerBlock), lds, s, L);
    return hipGetLastError();
}

template <class P, int PPL>
hipError_t launch_cls(const TrialLaunch &L, hipStream_t s) {
    if (L.n_items <= 0) return hipSuccess;
    return L.method == 0 ? launch_one<P, PPL, 0>(L, s) : launch_one<P, PPL, 1>(L, s);
}

template <class P>
hipError_t launch_policy(int cls, const TrialLaunch &L, hipStream_t s) {
    switch (kClassPPL[cls]) {
    case 1: return launch_cls<P, 1>(L, s);
    case 2: return launch_cls<P, 2>(L, s);
    case 3: return launch_cls<P, 3>(L, s);
    case 4: return launch_cls<P, 4>(L, s);
    case 6: return launch_cls<P, 6>(L, s);
    case 8: return launch_cls<P, 8>(L, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_trials_fp64(int cls, const TrialLaunch &L, hipStream_t s) {
    return launch_policy<F64>(cls, L, s);
}

hipError_t launch_trials_fp32c(int cls, const TrialLaunch &L, hipStream_t s) {
    return launch_policy<F32C>(cls, L, s);
}

}  // namespace ssg
