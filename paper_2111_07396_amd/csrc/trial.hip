// Fused per-trial kernel: fold -> LDS bucket sort -> Super Smoother (Listing
// 1) or the single-pass GCV variant (Sec. 3) -> chi^2 -> P -> tile argmax.
//
// One wavefront owns one (object, frequency tile) work item and runs its
// trials one after another; the object's points stay in registers, PPL
// consecutive sorted points per lane.  Arithmetic follows the policy P
// (numeric.hpp): FP64, or FP32 with compensated float-pair sums.
//
// Window sums of the running-line smoother come from prefix sums held in LDS.
// A window that wraps around the phase cycle is read from the periodic
// extension of the prefix sums (x shifted by +-1 on the far side), so every
// point costs the same two lookups per quantity.
#include "numeric.hpp"
#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

constexpr int kWavesPerBlock = 4;

template <int PPL>
struct Lay {
    static constexpr int NP = kWave * PPL;
    static constexpr int A8 = (NP + 1) * 8;
    // smoothing region: five prefix arrays of NP+1 eight-byte sums
    static constexpr int PW = 0, PX = A8, PXX = 2 * A8, PV = 3 * A8, PXV = 4 * A8;
    static constexpr int SMOOTH_END = 5 * A8;
    // sort region (aliases the smoothing region; dead once the sort is done)
    static constexpr int CNT = 0;
    static constexpr int TMP = ((NP + 1) * 4 + 15) / 16 * 16;
    static constexpr int SY = TMP + NP * 8;
    static constexpr int SW = SY + NP * 8;
    static constexpr int SORT_END = SW + NP * 8;
    // sorted keys live for the whole trial
    static constexpr int SK = ((SMOOTH_END > SORT_END ? SMOOTH_END : SORT_END) + 15) / 16 * 16;
    static constexpr int BYTES = SK + NP * 8;
};

template <class P>
struct Trial {
    using S = typename P::S;
    S *PW, *PX, *PXX, *PV, *PXV;
    const uint64_t *SK;
    int n, lane;
    S TW, TX, TXX;  // prefix totals of w, w x, w x^2
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
        S acc = P::zero();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            acc = p == 0 ? v[m][0] : P::add(acc, v[m][p]);
            loc[m][p] = acc;
        }
        tot[m] = acc;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        S excl = P::sub(P::scan(tot[m]), tot[m]);
#pragma unroll
        for (int p = 0; p < PPL; ++p) Pf[m][lane * PPL + p + 1] = P::add(excl, loc[m][p]);
        if (lane == 0) Pf[m][0] = P::zero();
    }
}

// q*T for q in {-1, 0, 1}
template <class P>
__device__ __forceinline__ typename P::S qmul(int q, typename P::S T) {
    return q > 0 ? T : (q < 0 ? P::neg(T) : P::zero());
}

// Periodic extension of the prefix sums at index i in [-n, 2n): q = floor(i/n)
// whole cycles, the far copies of x shifted by q.
template <class P>
struct ExtX {
    typename P::S w, x, xx;
};
template <class P>
__device__ __forceinline__ ExtX<P> ext_x(const Trial<P> &T, int i) {
    using S = typename P::S;
    const int q = (i < 0) ? -1 : (i >= T.n ? 1 : 0);
    const int r = i - q * T.n;
    S pw = T.PW[r], px = T.PX[r], pxx = T.PXX[r];
    ExtX<P> e;
    if (q == 0) {
        e.w = pw;
        e.x = px;
        e.xx = pxx;
        return e;
    }
    // q = +1: T + P(r) with x+1:   w: TW+pw        x: TX+px+pw     xx: TXX+pxx+2px+pw
    // q = -1: P(r) - T, x-1:       w: pw-TW        x: px-pw-TX+TW  xx: pxx-2px+pw-TXX+2TX-TW
    e.w = P::add(pw, qmul<P>(q, T.TW));
    S x = P::add(px, qmul<P>(q, P::add(pw, T.TX)));
    e.x = q < 0 ? P::add(x, T.TW) : x;
    S xx = P::add(pxx, P::add(qmul<P>(q, P::twice(px)), pw));
    xx = P::add(xx, qmul<P>(q, T.TXX));
    e.xx = q < 0 ? P::add(xx, P::sub(P::twice(T.TX), T.TW)) : xx;
    return e;
}

template <class P>
struct ExtV {
    typename P::S v, xv;
};
template <class P>
__device__ __forceinline__ ExtV<P> ext_v(const Trial<P> &T, int i, typename P::S TV,
                                         typename P::S TXV) {
    using S = typename P::S;
    const int q = (i < 0) ? -1 : (i >= T.n ? 1 : 0);
    const int r = i - q * T.n;
    S pv = T.PV[r], pxv = T.PXV[r];
    ExtV<P> e;
    if (q == 0) {
        e.v = pv;
        e.xv = pxv;
        return e;
    }
    // q = +1: v: TV+pv  xv: TXV+pxv+pv     q = -1: v: pv-TV  xv: pxv-pv-TXV+TV
    e.v = P::add(pv, qmul<P>(q, TV));
    S xv = P::add(pxv, qmul<P>(q, P::add(pv, TXV)));
    e.xv = q < 0 ? P::add(xv, TV) : xv;
    return e;
}

// Geometry of the window of point j (x-moments only).
template <class P>
struct XWin {
    typename P::S xm;  // weighted mean phase of the window
    typename P::R iW, iV, dx;
};
template <class P>
__device__ __forceinline__ XWin<P> xwin(const Trial<P> &T, int j, int b, typename P::S xj) {
    using R = typename P::R;
    ExtX<P> hi = ext_x<P>(T, j + b + 1), lo = ext_x<P>(T, j - b);
    auto W = P::sub(hi.w, lo.w), Sx = P::sub(hi.x, lo.x), Sxx = P::sub(hi.xx, lo.xx);
    XWin<P> g;
    g.iW = P::rcp(P::real(W));
    g.xm = P::quot(Sx, W, g.iW);
    const R V = P::real(P::sub(Sxx, P::mul(Sx, g.xm)));
    g.iV = (double)V > T.vsmlsq ? P::rcp(V) : R(0);
    g.dx = P::real(P::sub(xj, g.xm));
    return g;
}

// Fitted value of v at point j from the window sums of w v and w x v.
template <class P>
__device__ __forceinline__ typename P::R fit_at(const Trial<P> &T, const XWin<P> &g, int j, int b,
                                                typename P::S TV, typename P::S TXV) {
    using R = typename P::R;
    ExtV<P> hi = ext_v<P>(T, j + b + 1, TV, TXV), lo = ext_v<P>(T, j - b, TV, TXV);
    auto Sv = P::sub(hi.v, lo.v), Sxv = P::sub(hi.xv, lo.xv);
    const R vm = P::real(Sv) * g.iW;
    const R C = P::real(P::sub(Sxv, P::mul(g.xm, Sv)));
    return vm + C * g.iV * g.dx;
}

template <class P, int PPL>
__device__ __forceinline__ void set_prefix_v(Trial<P> &T, const typename P::S (&x)[PPL],
                                             const typename P::R (&w)[PPL],
                                             const typename P::R (&v)[PPL]) {
    using S = typename P::S;
    S q[2][PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        q[0][p] = P::prod(w[p], v[p]);
        q[1][p] = P::mul(q[0][p], x[p]);
    }
    S *const Pf[2] = {T.PV, T.PXV};
    build_prefix<P, PPL, 2>(Pf, q, T.lane);
}

// Replaces s over every run of equal phase by the run's weighted mean.  Uses
// the PV/PXV arrays as scratch (they must be dead when this is called).
template <class P, int PPL>
__device__ void tie_average(Trial<P> &T, const uint64_t (&xk)[PPL], const typename P::R (&w)[PPL],
                            typename P::R (&s)[PPL]) {
    using R = typename P::R;
    R *S1 = (R *)T.PV, *S2 = (R *)T.PXV;
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = T.lane * PPL + p;
        if (j < T.n) {
            S1[j] = s[p];
            S2[j] = w[p];
        }
    }
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = T.lane * PPL + p;
        if (j >= T.n) continue;
        uint64_t xj = xk[p] >> 16;
        bool tl = j > 0 && (T.SK[j - 1] >> 16) == xj;
        bool tr = j + 1 < T.n && (T.SK[j + 1] >> 16) == xj;
        if (!(tl || tr)) continue;
        int j0 = j, j1 = j;
        while (j0 > 0 && (T.SK[j0 - 1] >> 16) == xj) --j0;
        while (j1 + 1 < T.n && (T.SK[j1 + 1] >> 16) == xj) ++j1;
        double sws = 0.0, sw = 0.0;
        for (int i = j0; i <= j1; ++i) {
            sws += (double)S2[i] * (double)S1[i];
            sw += (double)S2[i];
        }
        s[p] = sw > 0.0 ? (R)(sws / sw) : R(0);
    }
    wave_lds_sync();
}

// One running-line smooth of v (prefix of v must be built).  With cv, r gets
// the leave-one-out residuals |v - s|/(1 - w h), repeating the previous
// point's value where 1 - w h <= 0.
template <class P, int PPL>
__device__ void smooth_eval(Trial<P> &T, int b, const uint64_t (&xk)[PPL],
                            const typename P::S (&x)[PPL], const typename P::R (&w)[PPL],
                            const typename P::R (&v)[PPL], bool cv, typename P::R (&s)[PPL],
                            typename P::R (&r)[PPL]) {
    using R = typename P::R;
    const auto TV = T.PV[T.n], TXV = T.PXV[T.n];
    bool bad = false;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = T.lane * PPL + p;
        s[p] = R(0);
        r[p] = R(0);
        if (j >= T.n) continue;
        XWin<P> g = xwin<P>(T, j, b, x[p]);
        s[p] = fit_at<P>(T, g, j, b, TV, TXV);
        if (cv) {
            R h = g.iW + g.dx * g.dx * g.iV;
            R d = R(1) - w[p] * h;
            if (d > R(0)) {
                r[p] = P::fabs_(v[p] - s[p]) * P::rcp(d);
            } else {
                r[p] = R(-1);
                bad = true;
            }
        }
    }
    if (cv && wave_ballot(bad) != 0) {
        R *S1 = (R *)T.PV;
        wave_lds_sync();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int j = T.lane * PPL + p;
            if (j < T.n) S1[j] = r[p];
        }
        wave_lds_sync();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int j = T.lane * PPL + p;
            if (j < T.n && r[p] < R(0)) {
                int i = j - 1;
                while (i >= 0 && S1[i] < R(0)) --i;
                r[p] = i >= 0 ? S1[i] : R(0);
            }
        }
        wave_lds_sync();
    }
    if (T.ties) tie_average<P, PPL>(T, xk, w, s);
}

template <class P, int PPL>
__device__ __forceinline__ void smooth(Trial<P> &T, int b, const uint64_t (&xk)[PPL],
                                       const typename P::S (&x)[PPL],
                                       const typename P::R (&w)[PPL],
                                       const typename P::R (&v)[PPL], bool cv,
                                       typename P::R (&s)[PPL], typename P::R (&r)[PPL]) {
    wave_lds_sync();
    set_prefix_v<P, PPL>(T, x, w, v);
    wave_lds_sync();
    smooth_eval<P, PPL>(T, b, xk, x, w, v, cv, s, r);
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
        int j = T.lane * PPL + p;
        if (j < T.n) {
            R d = y[p] - smo[p];
            acc = P::add(acc, P::prod(w[p] * d, d));
        }
    }
    return wave_sum(P::dbl(acc));
}

// Listing 1 on the sorted trial; returns chi^2.  The eight smooths run as one
// rolled loop over passes so that a single copy of the smoother is live:
//   passes 0, 2, 4: cross-validated smooth of y at the tweeter, midrange and
//                   woofer spans (fit kept, |CV residual| passed on);
//   passes 1, 3, 5: midrange smooth of that residual, per-point span choice;
//   pass 6:         midrange smooth of the chosen spans, then the blend;
//   pass 7:         tweeter smooth of the blend.
template <class P, int PPL>
__device__ double supersmoother(Trial<P> &T, const TrialLaunch &L, const uint64_t (&xk)[PPL],
                                const typename P::S (&x)[PPL], const typename P::R (&w)[PPL],
                                const typename P::R (&y)[PPL]) {
    using R = typename P::R;
    R cur[PPL], s[PPL], r[PPL];
    if (L.fixed_span > 0.0) {
        smooth<P, PPL>(T, halfwidth(T.n, L.fixed_span), xk, x, w, y, true, s, r);
        return wave_chi2<P, PPL>(T, w, y, s);
    }
    const int bk[3] = {halfwidth(T.n, L.span[0]), halfwidth(T.n, L.span[1]),
                       halfwidth(T.n, L.span[2])};
    const R sp0 = (R)L.span[0], sp1 = (R)L.span[1], sp2 = (R)L.span[2];
    R s0[PPL], s1[PPL], s2[PPL], resmin[PPL], sel[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        resmin[p] = R(1.0e20);
        sel[p] = R(0);
        cur[p] = y[p];
    }
#pragma unroll 1
    for (int pass = 0; pass < 8; ++pass) {
        const int k = pass >> 1;
        const bool primary = pass < 6 && (pass & 1) == 0;
        const int b = primary ? bk[k] : (pass == 7 ? bk[0] : bk[1]);
        smooth<P, PPL>(T, b, xk, x, w, cur, primary, s, r);
        if (primary) {
            if (k == 0) {
#pragma unroll
                for (int p = 0; p < PPL; ++p) s0[p] = s[p];
            } else if (k == 1) {
#pragma unroll
                for (int p = 0; p < PPL; ++p) s1[p] = s[p];
            } else {
#pragma unroll
                for (int p = 0; p < PPL; ++p) s2[p] = s[p];
            }
#pragma unroll
            for (int p = 0; p < PPL; ++p) cur[p] = r[p];
        } else if (pass < 6) {
            const R span_k = (R)L.span[k];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                if (s[p] < resmin[p]) {
                    resmin[p] = s[p];
                    sel[p] = span_k;
                }
            }
            if (pass == 5) {
                // bass enhancement against the woofer's smoothed residual
                const double alpha = L.alpha;
                if (alpha > 0.0 && alpha <= 10.0) {
                    const R ex = (R)(10.0 - alpha);
#pragma unroll
                    for (int p = 0; p < PPL; ++p) {
                        if (resmin[p] < s[p] && resmin[p] > R(0)) {
                            R tmp = resmin[p] / s[p];
                            if (tmp < R(1.0e-7)) tmp = R(1.0e-7);
                            sel[p] += (sp2 - sel[p]) * bass_pow<P>(tmp, ex);
                        }
                    }
                }
#pragma unroll
                for (int p = 0; p < PPL; ++p) cur[p] = sel[p];
            } else {
#pragma unroll
                for (int p = 0; p < PPL; ++p) cur[p] = y[p];
            }
        } else if (pass == 6) {
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                R sj = s[p];
                if (sj <= sp0) sj = sp0;
                if (sj >= sp2) sj = sp2;
                R f = sj - sp1;
                if (f < R(0)) {
                    f /= sp0 - sp1;
                    cur[p] = (R(1) - f) * s1[p] + f * s0[p];
                } else {
                    f /= sp2 - sp1;
                    cur[p] = (R(1) - f) * s1[p] + f * s2[p];
                }
            }
        }
    }
    return wave_chi2<P, PPL>(T, w, y, s);
}

// Sec. 3 single pass: one prefix of y serves every candidate span.
template <class P, int PPL>
__device__ double single_pass(Trial<P> &T, const TrialLaunch &L, const uint64_t (&xk)[PPL],
                              const typename P::S (&x)[PPL], const typename P::R (&w)[PPL],
                              const typename P::R (&y)[PPL]) {
    using R = typename P::R;
    const int K = L.fixed_span > 0.0 ? 1 : 3;
    wave_lds_sync();
    set_prefix_v<P, PPL>(T, x, w, y);
    wave_lds_sync();
    double best = 0.0, chi2 = 0.0;
    for (int k = 0; k < K; ++k) {
        const double span = L.fixed_span > 0.0 ? L.fixed_span : L.span[k];
        const int b = halfwidth(T.n, span);
        const auto TV = T.PV[T.n], TXV = T.PXV[T.n];
        R s[PPL], lev[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int j = T.lane * PPL + p;
            s[p] = R(0);
            lev[p] = R(0);
            if (j >= T.n) continue;
            XWin<P> g = xwin<P>(T, j, b, x[p]);
            s[p] = fit_at<P>(T, g, j, b, TV, TXV);
            lev[p] = g.iW + g.dx * g.dx * g.iV;
        }
        if (T.ties) {
            tie_average<P, PPL>(T, xk, w, s);
            if (k + 1 < K) {  // the tie scratch overwrote the prefix of y
                set_prefix_v<P, PPL>(T, x, w, y);
                wave_lds_sync();
            }
        }
        auto rss = P::zero(), tr = P::zero();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int j = T.lane * PPL + p;
            if (j < T.n) {
                R d = y[p] - s[p];
                rss = P::add(rss, P::prod(w[p] * d, d));
                tr = P::add(tr, P::prod(w[p], lev[p]));
            }
        }
        const double rss_d = wave_sum(P::dbl(rss));
        const double tr_d = wave_sum(P::dbl(tr));
        double gcv = __builtin_inf();
        if (tr_d < (double)T.n) {
            double den = 1.0 - tr_d / (double)T.n;
            gcv = rss_d / (den * den);
        }
        if (k == 0 || gcv < best) {
            best = gcv;
            chi2 = rss_d;
        }
    }
    return chi2;
}

template <class P, int PPL, int METHOD>
__device__ double run_trial(unsigned char *lds, int lane, int n, const TrialLaunch &L,
                            const double (&tt)[PPL], const typename P::R (&yv)[PPL],
                            const typename P::R (&wv)[PPL], double f, double chi0) {
    using R = typename P::R;
    using S = typename P::S;
    using Y = Lay<PPL>;
    constexpr int NP = Y::NP;
    // ---- fold (FP64): phase = frac(tt*f), as a 48-bit fixed-point key with
    // the point index in the low 16 bits (stable order on equal phases)
    uint64_t key[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = lane * PPL + p;
        if (j < n) {
            double u = tt[p] * f;
            double ph = u - floor(u);
            uint64_t ph48 = (uint64_t)(ph * 0x1p48);
            key[p] = (ph48 << 16) | (uint64_t)j;
        } else {
            key[p] = ~0ull;
        }
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
        int j = lane * PPL + p;
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
        uint32_t incl = wave_incl_sum_u32(tot);
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
        int j = lane * PPL + p;
        if (j < n) tmp[cnt[bkt[p]] + slot[p]] = key[p];
    }
    wave_lds_sync();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = lane * PPL + p;
        if (j < n) {
            uint32_t s = cnt[bkt[p]], e = cnt[bkt[p] + 1];
            uint32_t rank = 0;
            for (uint32_t i = s; i < e; ++i) rank += tmp[i] < key[p] ? 1u : 0u;
            uint32_t pos = s + rank;
            SK[pos] = key[p];
            sy[pos] = yv[p];
            sw[pos] = wv[p];
        }
    }
    wave_lds_sync();
    uint64_t xk[PPL];
    S x[PPL];
    R y[PPL], w[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = lane * PPL + p;
        if (j < n) {
            xk[p] = SK[j];
            y[p] = sy[j];
            w[p] = sw[j];
            x[p] = P::x_of_key(xk[p]);
        } else {
            xk[p] = ~0ull;
            y[p] = R(0);
            w[p] = R(0);
            x[p] = P::zero();
        }
    }
    wave_lds_sync();

    Trial<P> T;
    T.PW = (S *)(lds + Y::PW);
    T.PX = (S *)(lds + Y::PX);
    T.PXX = (S *)(lds + Y::PXX);
    T.PV = (S *)(lds + Y::PV);
    T.PXV = (S *)(lds + Y::PXV);
    T.SK = SK;
    T.n = n;
    T.lane = lane;

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
        bool tie = false;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            int j = lane * PPL + p;
            if (j + 1 < n) tie |= (SK[j + 1] >> 16) == (xk[p] >> 16);
        }
        T.ties = wave_ballot(tie) != 0;
    }
    // ---- x-moment prefix sums, shared by every smooth of this trial
    {
        S q[3][PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            q[0][p] = P::from(w[p]);
            q[1][p] = P::mulr(x[p], w[p]);
            q[2][p] = P::mul(q[1][p], x[p]);
        }
        S *const Pf[3] = {T.PW, T.PX, T.PXX};
        build_prefix<P, PPL, 3>(Pf, q, lane);
        wave_lds_sync();
        T.TW = T.PW[n];
        T.TX = T.PX[n];
        T.TXX = T.PXX[n];
    }
    const double chi2 = (METHOD == 0) ? supersmoother<P, PPL>(T, L, xk, x, w, y)
                                      : single_pass<P, PPL>(T, L, xk, x, w, y);
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
    const R *ysrc = P::kIsF64 ? (const R *)L.cat.yc : (const R *)L.cat.yc32;
    const R *wsrc = P::kIsF64 ? (const R *)L.cat.w : (const R *)L.cat.w32;
    double tt[PPL];
    R yv[PPL], wv[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        int j = lane * PPL + p;
        bool ok = j < n;
        tt[p] = ok ? L.cat.tt[base + j] : 0.0;
        yv[p] = ok ? ysrc[base + j] : R(0);
        wv[p] = ok ? wsrc[base + j] : R(0);
    }
    const double chi0 = L.cat.chi0[obj];
    double best_p = 0.0;
    int32_t best_k = -1;
    for (int64_t k = k0; k < k1; ++k) {
        const double f = grid_freq(L.fmin, L.df, k);
        const double Pk = run_trial<P, PPL, METHOD>(lds, lane, n, L, tt, yv, wv, f, chi0);
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
