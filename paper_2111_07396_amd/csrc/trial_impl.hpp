// Fused per-trial kernel (templates; instantiated per precision policy in
// trial_f64.hip and trial_f32c.hip): fold -> LDS bucket sort -> Super Smoother (Listing
// 1) or the single-pass variant (Sec. 3, two readings) -> chi^2 -> P ->
// running argmax of the work item.
//
// A trial group of NW wavefronts (one workgroup) owns one (object, frequency
// tile) work item and runs its trials one after another; thread t of the
// group holds the PPL consecutive sorted points t*PPL .. t*PPL+PPL-1.
// Arithmetic follows the policy P (numeric.hpp): FP64, or FP32 with
// compensated float-pair sums.
//
// Every running-line smooth is a pair of window sums (of w v and w x v)
// combined with the window's geometry (numeric.hpp, Geo), which depends only
// on the sorted phases and the span.  Window sums are differences of prefix
// sums kept in LDS together with their periodic extension: the prefix is
// continued for `ext` slots past both ends with the far copies of the phase
// shifted by +-1, so the window [j-b, j+b] is always P[j+b+1] - P[j-b].
//   phase A1: prefix of w, w x, w x^2 -> geometry of every span;
//   phase A2: prefix of w y, w x y    -> the cross-validated smooths of y;
//   phase B:  one prefix pair per later smooth (residuals, spans, blend).
// The prefixes of one slot are stored together (F values per slot, see
// qaddr), so that one LDS address serves every prefix a window end needs.
#pragma once
#include "numeric.hpp"
#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

// ------------------------------------------------------------------ layout
// Prefix storage: slot u holds F consecutive values: the x-moment prefixes
// (W, X, XX) in fields 0..2 during the geometry phase, then a prefix pair
// (V, XV) in fields 0, 1.  Double-buffered groups (F = 5) hold the prefix
// pair of y in fields 3, 4 beside the x-moments (phases A1 and A2 share one
// pass), and alternate their later pairs between fields (0, 1) and (2, 3).
// A window end is then one address with constant offsets (paired loads)
// instead of one address per prefix array.
// After every PPL slots come pad_q values: the 64 lanes read at a common
// offset from their own PPL consecutive slots, and the pad makes the lane
// stride an odd number of 8-byte words (F = 3) or of 16-byte words (F = 4),
// so that the lanes of one LDS cycle fall in distinct banks.
constexpr __host__ __device__ int pad_q(int f, int ppl) {
    return f == 4 ? 2 : ((f * ppl) % 2 == 0 ? 1 : 0);
}
template <int F, int PPL>
__host__ __device__ __forceinline__ int qaddr(int u) {
    return u * F + (u / PPL) * pad_q(F, PPL);
}

// Groups of up to 1,024 points keep the work item's object (t, y, w) in LDS
// for all of its trials; larger groups read it from global memory per trial
// and carry y, w through the sort.
constexpr __host__ __device__ bool caches_object(int np) { return np <= 1024; }

// Prefix arrays of a trial group.  The SS kernels of multi-wavefront groups
// that cache the object alternate their later smooths between two prefix
// pairs, fields (0, 1) and (2, 3) of the prefix slots: a pass then needs no
// barrier before it
// writes, as the pair it overwrites was last read two passes earlier, behind
// that pass's barriers (measured: +3-7 % on these kernels; a single
// wavefront's barrier is only a wait on its own LDS operations, and there the
// change lost up to 9 %).
constexpr __host__ __device__ bool double_buffered(int method, int nw, int ppl) {
    return method == 0 && nw > 1 && caches_object(kWave * nw * ppl);
}
constexpr __host__ __device__ int prefix_arrays(int method, int nw, int ppl) {
    return double_buffered(method, nw, ppl) ? 5 : 3;
}

// Bucket members that the sort's ranking loads at once per slot.  With as
// many buckets as slots most buckets hold at most this many keys (measured:
// 4 beats 2, 6 and 8).  The ranking reads bucketed keys up to index
// n + kRankU - 1, inside the prefix region (at least 3 np values).
constexpr int kRankU = 4;

// LDS layout of one trial group; identical on host and device.  The prefix
// region starts at 0 and also serves as scratch of three arrays of np values
// (tie averaging, CV fallbacks), and as the sort's bucketed keys.  The sort's
// bucket counters have a region of their own, kept zero between trials.
struct Layout {
    int np, ext, F, qbytes, sk, xch, qslot, best, obj, cnt, bytes;
    __host__ __device__ Layout(int nw, int ppl, int ext_, int method) {
        np = kWave * nw * ppl;
        ext = ext_;
        F = prefix_arrays(method, nw, ppl);
        const bool cache = caches_object(np);
        const int ulen = np + 2 * ext + 1;
        int nd = (ulen - 1) * F + ((ulen - 1) / ppl) * pad_q(F, ppl) + F;  // values
        if (nd < 3 * np) nd = 3 * np;
        qbytes = (nd * 8 + 15) / 16 * 16;
        const int sort_end = (cache ? 1 : 3) * np * 8;
        int a = qbytes > sort_end ? qbytes : sort_end;
        sk = (a + 15) / 16 * 16;
        xch = sk + np * 8;
        qslot = xch + nw * 8 * 8;
        best = qslot + 16;
        obj = best + kMaxSharedBatch * 12;
        cnt = obj + (cache ? 3 * np * 8 : 0);
        bytes = cnt + ((np + 1) * 4 + 15) / 16 * 16;
    }
};

// A value loaded at a wave-uniform address, made a scalar (so that the
// addresses formed from it live in scalar registers).
__device__ __forceinline__ int uniform_i32(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform_i64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

template <class T>
__device__ __forceinline__ const T *uniform_ptr(const T *p) {
    return (const T *)uniform_i64((int64_t)p);
}

template <int NW>
__device__ __forceinline__ void bsync() {
    if constexpr (NW == 1) {
        wave_lds_sync();
    } else {
        __syncthreads();
    }
}

template <class P, int NW, int PPL, int F>
struct Group {
    using S = typename P::S;
    static constexpr int NT = kWave * NW;
    S *Q;                    // interleaved prefix storage (or scratch)
    const uint64_t *SK;      // sorted keys
    S *xs;                   // exchange slots for group scans
    double *xd;              // exchange slots for group sums
    int t, wave, lane, n, ext;
    int hw[3], hwf;          // half-widths of the spans and of the fixed span at n
    typename P::R ilo, ihi;  // 1/(span0 - span1), 1/(span2 - span1) of the blend
    double vsmlsq;
    double inv_n, inv_chi0;  // 1/n and 1/chi0 of the work item's object
    bool ties;
    mutable typename P::Z z;  // cross-row scan temporaries (see wave_incl_sum_z)
    // first value of prefix slot i (i = -ext .. n + ext)
    __device__ int at(int i) const { return qaddr<F, PPL>(ext + i); }
    // scratch array k (0..2) of NT * PPL values of type R
    template <class R>
    __device__ R *scratch(int k) const { return (R *)Q + k * (NT * PPL); }
};

// Half-window of a span: b = max(2, floor(0.5*span*n + 0.5)), clamped so
// that 2b+1 <= n.
__host__ __device__ __forceinline__ int halfwidth(int n, double span) {
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

// ------------------------------------------------------------------ group reductions
// Sum over the wavefront (all lanes active), identical in every lane.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ double wave_total(const Group<P, NW, PPL, F> &G, double a) {
    if constexpr (P::kIsF64) {
        return readlane_f64(wave_incl_sum_z(a, G.z.z15, G.z.z31), kWave - 1);
    } else {
        return wave_sum(a);
    }
}

// Sum over the group of one double, identical in every thread.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ double group_sum1(const Group<P, NW, PPL, F> &G, double a) {
    a = wave_total(G, a);
    if constexpr (NW > 1) {
        if (G.lane == 0) G.xd[G.wave] = a;
        __syncthreads();
        a = 0.0;
        for (int w = 0; w < NW; ++w) a += G.xd[w];
        __syncthreads();
    }
    return a;
}

// The same for the last reduction of a trial (its chi^2): exchange slots of
// their own (3 NW .. 4 NW, used by nothing else) and no trailing barrier -- the
// next writer of these slots is the next trial's chi^2 sum, behind the
// barriers of its sort and smoother.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ double group_sum1_last(const Group<P, NW, PPL, F> &G, double a) {
    a = wave_total(G, a);
    if constexpr (NW > 1) {
        double *x = G.xd + 3 * NW;
        if (G.lane == 0) x[G.wave] = a;
        __syncthreads();
        a = 0.0;
        for (int w = 0; w < NW; ++w) a += x[w];
    }
    return a;
}

// Sum over the group of two doubles, identical in every thread.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void group_sum2(const Group<P, NW, PPL, F> &G, double &a, double &b) {
    a = wave_total(G, a);
    b = wave_total(G, b);
    if constexpr (NW > 1) {
        if (G.lane == 0) {
            G.xd[2 * G.wave] = a;
            G.xd[2 * G.wave + 1] = b;
        }
        __syncthreads();
        a = 0.0;
        b = 0.0;
        for (int w = 0; w < NW; ++w) {
            a += G.xd[2 * w];
            b += G.xd[2 * w + 1];
        }
        __syncthreads();
    }
}

// Exclusive prefix over the group's threads of M values; also the totals.
// XO: first exchange slot (consecutive builds without a barrier between them
// use disjoint slots).
template <class P, int NW, int PPL, int M, int F, int XO = 0>
__device__ __forceinline__ void group_excl(const Group<P, NW, PPL, F> &G,
                                           const typename P::S (&tot)[M],
                                           typename P::S (&excl)[M], typename P::S (&all)[M]) {
    using S = typename P::S;
    S *const xs = G.xs + XO;
    S incl[M];
    P::template scan_n<M>(tot, incl, G.z);
    if constexpr (NW == 1) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
            excl[m] = P::sub(incl[m], tot[m]);
            all[m] = P::lane_value(incl[m], kWave - 1);
        }
    } else {
        if (G.lane == kWave - 1) {
#pragma unroll
            for (int m = 0; m < M; ++m) xs[m * NW + G.wave] = incl[m];
        }
        __syncthreads();
#pragma unroll
        for (int m = 0; m < M; ++m) {
            if constexpr (NW == 2 && P::kIsF64) {
                // the first wavefront's total is added by the second only:
                // an FMA with the (wave-uniform) factor 1 or 0 is that add
                // exactly, or nothing
                const S v0 = xs[m * 2], v1 = xs[m * 2 + 1];
                excl[m] = fma(v0, G.wave ? 1.0 : 0.0, incl[m] - tot[m]);
                all[m] = v0 + v1;
            } else {
                S off = P::zero(), sum = P::zero();
                for (int w = 0; w < NW; ++w) {
                    const S v = xs[m * NW + w];
                    if (w < G.wave) off = P::add(off, v);
                    sum = P::add(sum, v);
                }
                excl[m] = P::add(off, P::sub(incl[m], tot[m]));
                all[m] = sum;
            }
        }
    }
}

// Exclusive prefix sums P[i] = sum_{j<i} v_j of M quantities at slots
// 0..n (padding points contribute 0); returns the totals.  Ends with a sync
// (TRAIL; without it a later build's barrier must order the writes).
// EXT: the arrays are the x-moment prefix (W, X, XX; M = 3) or a prefix pair
// (V, XV of w v and w x v; M = 2), and their periodic extension by e slots
// per side is written with them: each thread writes the copies of its own
// prefix values (every thread holds the totals after the group scan).
//   right: P(n+k) = T + P(k)   with the copy's phase shifted by +1,
//   left:  P(-k) = P(n-k) - T  with the copy's phase shifted by -1,
// so that X and XX pick up the terms of (x +- 1) and (x +- 1)^2.  Slots past
// n + e are left unwritten (no window reaches them).
template <class P, int NW, int PPL, int M, bool EXT, int F, bool TRAIL = true, int XO = 0>
__device__ __forceinline__ void build_prefix(const Group<P, NW, PPL, F> &G,
                                             typename P::S *const (&Pf)[M],
                                             const typename P::S (&v)[M][PPL],
                                             typename P::S (&T)[M], int e = 0) {
    static_assert(!EXT || M == 2 || M == 3, "extension of a pair or of the x-moments");
    using S = typename P::S;
    S loc[M][PPL], tot[M], excl[M];
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
    group_excl<P, NW, PPL, M, F, XO>(G, tot, excl, T);
    const int n = G.n;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int u = G.t * PPL + p + 1;
        S val[M];
#pragma unroll
        for (int m = 0; m < M; ++m) val[m] = P::add(excl[m], loc[m][p]);
        if (!EXT || u <= n) {
#pragma unroll
            for (int m = 0; m < M; ++m) Pf[m][G.at(u)] = val[m];
        }
        if constexpr (EXT) {
            if (u <= e && u <= n) {  // right copy, k = u
                const int d = G.at(n + u);
                if constexpr (M == 3) {
                    Pf[0][d] = P::add(T[0], val[0]);
                    Pf[1][d] = P::add(P::add(T[1], val[1]), val[0]);
                    Pf[2][d] = P::add(P::add(T[2], val[2]), P::add(P::twice(val[1]), val[0]));
                } else {
                    Pf[0][d] = P::add(T[0], val[0]);
                    Pf[1][d] = P::add(P::add(T[1], val[1]), val[0]);
                }
            }
            if (u < n && u >= n - e) {  // left copy, k = n - u
                const int d = G.at(u - n);
                if constexpr (M == 3) {
                    const S rw = P::sub(T[0], val[0]);
                    const S rx = P::sub(T[1], val[1]);
                    const S rxx = P::sub(T[2], val[2]);
                    Pf[0][d] = P::neg(rw);
                    Pf[1][d] = P::sub(rw, rx);
                    Pf[2][d] = P::neg(P::add(P::sub(rxx, P::twice(rx)), rw));
                } else {
                    const S rv = P::sub(T[0], val[0]);
                    const S rxv = P::sub(T[1], val[1]);
                    Pf[0][d] = P::neg(rv);
                    Pf[1][d] = P::sub(rv, rxv);
                }
            }
        }
    }
    if (G.t == 0) {
#pragma unroll
        for (int m = 0; m < M; ++m) Pf[m][G.at(0)] = P::zero();
    }
    if constexpr (TRAIL) bsync<NW>();
}

// Periodic extension of the x-moment prefix (W, X, XX) by e slots per side.
// Right: P(n+k) = T + P(k) with the copy's phase shifted by +1.
// Left:  P(-k) = P(n-k) - T with the copy's phase shifted by -1.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void extend3(const Group<P, NW, PPL, F> &G, typename P::S *W,
                                        typename P::S *X, typename P::S *XX,
                                        const typename P::S (&T)[3], int e) {
    const int n = G.n;
    for (int q = G.t; q < 2 * e; q += Group<P, NW, PPL, F>::NT) {
        if (q < e) {
            const int k = q + 1;
            const auto pw = W[G.at(k)], px = X[G.at(k)], pxx = XX[G.at(k)];
            const int d = G.at(n + k);
            W[d] = P::add(T[0], pw);
            X[d] = P::add(P::add(T[1], px), pw);
            XX[d] = P::add(P::add(T[2], pxx), P::add(P::twice(px), pw));
        } else {
            const int k = q - e + 1;
            const auto rw = P::sub(T[0], W[G.at(n - k)]);
            const auto rx = P::sub(T[1], X[G.at(n - k)]);
            const auto rxx = P::sub(T[2], XX[G.at(n - k)]);
            const int d = G.at(-k);
            W[d] = P::neg(rw);
            X[d] = P::sub(rw, rx);
            XX[d] = P::neg(P::add(P::sub(rxx, P::twice(rx)), rw));
        }
    }
    bsync<NW>();
}

// Same for a prefix pair (V, XV) of w v and w x v.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void extend2(const Group<P, NW, PPL, F> &G, typename P::S *V,
                                        typename P::S *XV, const typename P::S (&T)[2], int e) {
    const int n = G.n;
    for (int q = G.t; q < 2 * e; q += Group<P, NW, PPL, F>::NT) {
        if (q < e) {
            const int k = q + 1;
            const auto pv = V[G.at(k)], pxv = XV[G.at(k)];
            const int d = G.at(n + k);
            V[d] = P::add(T[0], pv);
            XV[d] = P::add(P::add(T[1], pxv), pv);
        } else {
            const int k = q - e + 1;
            const auto rv = P::sub(T[0], V[G.at(n - k)]);
            const auto rxv = P::sub(T[1], XV[G.at(n - k)]);
            const int d = G.at(-k);
            V[d] = P::neg(rv);
            XV[d] = P::sub(rv, rxv);
        }
    }
    bsync<NW>();
}

// Whether a kernel writes the periodic extension inside the prefix build
// (one barrier less per prefix pass, a few more live registers) or in a
// separate pass (extend3 / extend2).  Measured on MI355X per shape (FP64):
// the fused form wins for one point per thread (up to 20 %) and for groups
// of several wavefronts at two points per thread (5-10 %); with more points
// per thread it raises the register peak and loses (up to 39 %).  The
// compensated-FP32 kernels, with twice the registers per sum, keep the
// separate pass.
template <bool F64, int NW, int PPL>
constexpr bool fused_extension() {
    return F64 && (PPL == 1 || (PPL == 2 && NW > 1));
}

// Prefix pair of w v and w x v, extended by e.  BUF 0: into fields (0, 1)
// after a barrier; BUF 1: into fields (2, 3), BUF 2: into (0, 1), both
// without one
// (double-buffered passes).
template <class P, int NW, int PPL, int BUF = 0, int F>
__device__ __forceinline__ void prefix_pair(const Group<P, NW, PPL, F> &G,
                                            const typename P::R (&w)[PPL],
                                            const typename P::S (&wx)[PPL],
                                            const typename P::R (&v)[PPL], int e) {
    using S = typename P::S;
    S q[2][PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        q[0][p] = P::prod(w[p], v[p]);
        q[1][p] = P::mulr(wx[p], v[p]);
    }
    S *const V = G.Q + (BUF == 1 ? 2 : 0);
    S *const XV = V + 1;
    S *const Pf[2] = {V, XV};
    S T[2];
    if constexpr (BUF == 0) bsync<NW>();
    if constexpr (fused_extension<P::kIsF64, NW, PPL>()) {
        build_prefix<P, NW, PPL, 2, true>(G, Pf, q, T, e);
    } else {
        build_prefix<P, NW, PPL, 2, false>(G, Pf, q, T);
        extend2<P, NW, PPL>(G, V, XV, T, e);
    }
}

template <class P, int NW, int PPL, int F>
__device__ __forceinline__ typename P::Geo geometry(const Group<P, NW, PPL, F> &G, int j, int b,
                                                    typename P::S xj, typename P::R &h) {
    const int hi = G.at(j + b + 1), lo = G.at(j - b);
    const typename P::S *Q = G.Q;
    return P::geo(P::sub(Q[hi], Q[lo]), P::sub(Q[hi + 1], Q[lo + 1]), P::sub(Q[hi + 2], Q[lo + 2]),
                  xj, G.vsmlsq, h);
}

// Fit of the prefix pair in fields (OFF, OFF + 1) at point j, half-width b.
template <class P, int NW, int PPL, int F, int OFF = 0>
__device__ __forceinline__ typename P::R window_fit(const Group<P, NW, PPL, F> &G,
                                                    const typename P::Geo &g, int j, int b) {
    const int hi = G.at(j + b + 1) + OFF, lo = G.at(j - b) + OFF;
    const typename P::S *Q = G.Q;
    return P::eval(g, P::sub(Q[hi], Q[lo]), P::sub(Q[hi + 1], Q[lo + 1]));
}

// ------------------------------------------------------------------ rare paths
// Kept out of line; they work on LDS only, so no register arrays cross the
// call.  One copy per kernel (the TAG template argument): a function shared by
// kernels of different register budgets is compiled for the tightest of
// them, and the callers' register allocation then depends on the other
// kernels in the file.

// out[j] (j in [j0, j1)) = weighted mean of s over the run of equal phase
// holding j, or s[j] when the phase of j is unique.
template <class R, int TAG>
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
template <class R, int TAG>
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

// Replaces s over every run of equal phase by the run's weighted mean (the
// prefix storage is used as scratch and must be dead).
template <class P, int NW, int PPL, int F>
__device__ void tie_average(const Group<P, NW, PPL, F> &G, const typename P::R (&w)[PPL],
                            typename P::R (&s)[PPL]) {
    using R = typename P::R;
    R *S1 = G.template scratch<R>(0), *S2 = G.template scratch<R>(1),
      *S3 = G.template scratch<R>(2);
    bsync<NW>();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = G.t * PPL + p;
        if (j < G.n) {
            S1[j] = s[p];
            S2[j] = w[p];
        }
    }
    bsync<NW>();
    tie_means<R, (NW * 8 + PPL) * 8 + F>(S1, S2, S3, G.SK, G.n, min(G.t * PPL, G.n),
                                         min(G.t * PPL + PPL, G.n));
    bsync<NW>();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = G.t * PPL + p;
        if (j < G.n) s[p] = S3[j];
    }
    bsync<NW>();
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
// Uses the prefix storage as scratch.  `any` must be uniform over the group.
template <class P, int NW, int PPL, int F>
__device__ void cv_fallback(const Group<P, NW, PPL, F> &G, bool any, typename P::R (&r)[PPL]) {
    using R = typename P::R;
    if (!any) return;
    R *S1 = G.template scratch<R>(1), *S2 = G.template scratch<R>(2);
    bsync<NW>();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = G.t * PPL + p;
        if (j < G.n) S1[j] = r[p];
    }
    bsync<NW>();
    fallback_fill<R, (NW * 8 + PPL) * 8 + F>(S1, S2, min(G.t * PPL, G.n),
                                             min(G.t * PPL + PPL, G.n));
    bsync<NW>();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = G.t * PPL + p;
        if (j < G.n) r[p] = S2[j];
    }
    bsync<NW>();
}

// Whether any point of the group has a negative (marked) residual.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ bool group_any_neg(const Group<P, NW, PPL, F> &G,
                                              const typename P::R (&r)[PPL]) {
    bool bad = false;
#pragma unroll
    for (int p = 0; p < PPL; ++p) bad |= (G.t * PPL + p < G.n) && r[p] < typename P::R(0);
    if constexpr (NW == 1) {
        return wave_ballot(bad) != 0;
    } else {
        return __syncthreads_or(bad) != 0;
    }
}

// Weighted residual sum, accumulated per thread in the policy's sum type and
// reduced across the group in FP64.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ double chi2_of(const Group<P, NW, PPL, F> &G,
                                          const typename P::R (&w)[PPL],
                                          const typename P::R (&y)[PPL],
                                          const typename P::R (&smo)[PPL]) {
    using R = typename P::R;
    auto acc = P::zero();
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const R d = G.t * PPL + p < G.n ? y[p] - smo[p] : R(0);
        acc = P::add(acc, P::prod(w[p] * d, d));
    }
    return group_sum1_last<P, NW, PPL>(G, P::dbl(acc));
}

// Smooth of v with a stored geometry (phase B): prefix pair (BUF as in
// prefix_pair), fit, ties.
template <class P, int NW, int PPL, int BUF = 0, int F>
__device__ __forceinline__ void smooth_with(const Group<P, NW, PPL, F> &G, int b,
                                           const typename P::Geo (&g)[PPL],
                                           const typename P::R (&w)[PPL],
                                           const typename P::S (&wx)[PPL],
                                           const typename P::R (&v)[PPL], int e,
                                           typename P::R (&s)[PPL]) {
    prefix_pair<P, NW, PPL, BUF>(G, w, wx, v, e);
    const typename P::S *V = G.Q + (BUF == 1 ? 2 : 0);
    const typename P::S *XV = V + 1;
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = min(G.t * PPL + p, G.n - 1);
        const int hi = G.at(j + b + 1), lo = G.at(j - b);
        s[p] = P::eval(g[p], P::sub(V[hi], V[lo]), P::sub(XV[hi], XV[lo]));
    }
    if (G.ties) tie_average<P, NW, PPL>(G, w, s);
}

// Phase A1: prefix of the x-moments, extended by e.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void prefix_x(const Group<P, NW, PPL, F> &G,
                                         const typename P::S (&x)[PPL],
                                         const typename P::R (&w)[PPL],
                                         const typename P::S (&wx)[PPL], int e) {
    using S = typename P::S;
    S q[3][PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        q[0][p] = P::from(w[p]);
        q[1][p] = wx[p];
        q[2][p] = P::mul(wx[p], x[p]);
    }
    S *const Pf[3] = {G.Q, G.Q + 1, G.Q + 2};
    S T[3];
    bsync<NW>();
    if constexpr (fused_extension<P::kIsF64, NW, PPL>()) {
        build_prefix<P, NW, PPL, 3, true>(G, Pf, q, T, e);
    } else {
        build_prefix<P, NW, PPL, 3, false>(G, Pf, q, T);
        extend3<P, NW, PPL>(G, G.Q, G.Q + 1, G.Q + 2, T, e);
    }
}

// Phases A1 and A2 in one pass (five prefix fields per slot): the x-moment
// prefixes W, X, XX in fields 0..2 and the prefix pair of y in fields 3, 4,
// extended by e (two group scans of 3 and 2 quantities: one scan of all
// five holds more registers at once).  With the extension written inside
// the builds, the first build needs no trailing barrier (nothing reads its
// prefixes before the second build's), and the second exchanges its totals
// in slots of its own.
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void prefix_xy(const Group<P, NW, PPL, F> &G,
                                          const typename P::S (&x)[PPL],
                                          const typename P::R (&w)[PPL],
                                          const typename P::S (&wx)[PPL],
                                          const typename P::R (&y)[PPL], int e) {
    static_assert(F >= 5, "five prefix fields");
    using S = typename P::S;
    constexpr bool kFused = fused_extension<P::kIsF64, NW, PPL>();
    bsync<NW>();
    {
        S q[3][PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            q[0][p] = P::from(w[p]);
            q[1][p] = wx[p];
            q[2][p] = P::mul(wx[p], x[p]);
        }
        S *const Pf[3] = {G.Q, G.Q + 1, G.Q + 2};
        S T[3];
        build_prefix<P, NW, PPL, 3, kFused, F, !kFused>(G, Pf, q, T, e);
        if constexpr (!kFused) extend3<P, NW, PPL>(G, G.Q, G.Q + 1, G.Q + 2, T, e);
    }
    {
        S q[2][PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            q[0][p] = P::prod(w[p], y[p]);
            q[1][p] = P::mulr(wx[p], y[p]);
        }
        S *const Pf[2] = {G.Q + 3, G.Q + 4};
        S T[2];
        build_prefix<P, NW, PPL, 2, kFused, F, true, 4 * NW>(G, Pf, q, T, e);
        if constexpr (!kFused) extend2<P, NW, PPL>(G, G.Q + 3, G.Q + 4, T, e);
    }
}

// ------------------------------------------------------------------ Listing 1
template <class P, int NW, int PPL, int F>
__device__ double supersmoother(const Group<P, NW, PPL, F> &G, const TrialLaunch &L,
                                const typename P::S (&x)[PPL], const typename P::R (&w)[PPL],
                                const typename P::S (&wx)[PPL], const typename P::R (&y)[PPL],
                                const typename P::R *ysrc) {
    using R = typename P::R;
    using Geo = typename P::Geo;
    const int n = G.n, t = G.t;
    if (L.fixed_span > 0.0) {  // Listing 1: one smooth at the fixed span
        const int b = G.hwf;
        Geo g[PPL];
        R smo[PPL];
        prefix_x<P, NW, PPL>(G, x, w, wx, b);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            R h;
            g[p] = geometry<P, NW, PPL>(G, min(t * PPL + p, n - 1), b, x[p], h);
        }
        smooth_with<P, NW, PPL>(G, b, g, w, wx, y, b, smo);
        return chi2_of<P, NW, PPL>(G, w, y, smo);
    }
    const int b0 = G.hw[0], b1 = G.hw[1], b2 = G.hw[2];
    const R sp0 = (R)L.span[0], sp1 = (R)L.span[1], sp2 = (R)L.span[2];

    Geo g0[PPL], g1[PPL];
    R s0[PPL], s1[PPL], s2[PPL], r0[PPL], r1[PPL], r2[PPL];
    if constexpr (F >= 5) {
        // ---- phases A1 + A2 in one pass, span by span: geometry, fit and
        // |CV residual|; only the geometries used later stay live
        prefix_xy<P, NW, PPL>(G, x, w, wx, y, b2);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = min(t * PPL + p, n - 1);
            R h;
            const Geo g2 = geometry<P, NW, PPL>(G, j, b2, x[p], h);
            s2[p] = window_fit<P, NW, PPL, F, 3>(G, g2, j, b2);
            r2[p] = cv_resid<P>(y[p], s2[p], w[p], h);
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = min(t * PPL + p, n - 1);
            R h;
            g1[p] = geometry<P, NW, PPL>(G, j, b1, x[p], h);
            s1[p] = window_fit<P, NW, PPL, F, 3>(G, g1[p], j, b1);
            r1[p] = cv_resid<P>(y[p], s1[p], w[p], h);
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = min(t * PPL + p, n - 1);
            R h;
            g0[p] = geometry<P, NW, PPL>(G, j, b0, x[p], h);
            s0[p] = window_fit<P, NW, PPL, F, 3>(G, g0[p], j, b0);
            r0[p] = cv_resid<P>(y[p], s0[p], w[p], h);
        }
    } else {
        // ---- phase A1: geometry of the three spans
        Geo g2[PPL];
        R h0[PPL], h1[PPL], h2[PPL];
        prefix_x<P, NW, PPL>(G, x, w, wx, b2);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = min(t * PPL + p, n - 1);
            g0[p] = geometry<P, NW, PPL>(G, j, b0, x[p], h0[p]);
            g1[p] = geometry<P, NW, PPL>(G, j, b1, x[p], h1[p]);
            g2[p] = geometry<P, NW, PPL>(G, j, b2, x[p], h2[p]);
        }
        // ---- phase A2: the cross-validated smooths of y and their |CV residuals|
        prefix_pair<P, NW, PPL>(G, w, wx, y, b2);
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = min(t * PPL + p, n - 1);
            s0[p] = window_fit<P, NW, PPL>(G, g0[p], j, b0);
            s1[p] = window_fit<P, NW, PPL>(G, g1[p], j, b1);
            s2[p] = window_fit<P, NW, PPL>(G, g2[p], j, b2);
            r0[p] = cv_resid<P>(y[p], s0[p], w[p], h0[p]);
            r1[p] = cv_resid<P>(y[p], s1[p], w[p], h1[p]);
            r2[p] = cv_resid<P>(y[p], s2[p], w[p], h2[p]);
        }
    }
    // ---- phase B: fallbacks and ties of the primaries
    constexpr bool kDB = double_buffered(0, NW, PPL);
    if constexpr (kDB) {
        // one group vote for the three residual arrays (a fallback leaves an
        // array without marked residuals unchanged)
        bool bad = false;
#pragma unroll
        for (int p = 0; p < PPL; ++p)
            bad |= (t * PPL + p < n) && (r0[p] < R(0) || r1[p] < R(0) || r2[p] < R(0));
        const bool any_neg = __syncthreads_or(bad) != 0;
        cv_fallback<P, NW, PPL>(G, any_neg, r0);
        cv_fallback<P, NW, PPL>(G, any_neg, r1);
        cv_fallback<P, NW, PPL>(G, any_neg, r2);
    } else {
        cv_fallback<P, NW, PPL>(G, group_any_neg<P, NW, PPL>(G, r0), r0);
        cv_fallback<P, NW, PPL>(G, group_any_neg<P, NW, PPL>(G, r1), r1);
        cv_fallback<P, NW, PPL>(G, group_any_neg<P, NW, PPL>(G, r2), r2);
    }
    if (G.ties) {
        tie_average<P, NW, PPL>(G, w, s0);
        tie_average<P, NW, PPL>(G, w, s1);
        tie_average<P, NW, PPL>(G, w, s2);
    }
    // midrange smooths of the residuals; per-point span choice, the lowest
    // span winning ties (Listing 1 scans the spans upward with a strict <,
    // starting from 1e20; the span stays 0 if no residual is below that)
    // (double-buffered groups alternate the prefix pairs of these passes)
    constexpr int kB1 = kDB ? 1 : 0, kB2 = kDB ? 2 : 0;
    const int eb = b1 > b0 ? b1 : b0;
    R resmin[PPL], sel[PPL], rt[PPL];
    smooth_with<P, NW, PPL, kB1>(G, b1, g1, w, wx, r0, eb, rt);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const bool lt = rt[p] < R(1.0e20);
        resmin[p] = lt ? rt[p] : R(1.0e20);
        sel[p] = lt ? sp0 : R(0);
    }
    smooth_with<P, NW, PPL, kB2>(G, b1, g1, w, wx, r1, eb, rt);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const bool lt = rt[p] < resmin[p];
        resmin[p] = lt ? rt[p] : resmin[p];
        sel[p] = lt ? sp1 : sel[p];
    }
    smooth_with<P, NW, PPL, kB1>(G, b1, g1, w, wx, r2, eb, rt);
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
                R tmp = resmin[p] * P::rcp(rt[p]);
                if (tmp < R(1.0e-7)) tmp = R(1.0e-7);
                sel[p] += (sp2 - sel[p]) * bass_pow<P>(tmp, ex);
            }
        }
    }
    // midrange smooth of the chosen spans, clip, blend
    smooth_with<P, NW, PPL, kB2>(G, b1, g1, w, wx, sel, eb, rt);
    const R ilo = G.ilo, ihi = G.ihi;
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
    smooth_with<P, NW, PPL, kB1>(G, b0, g0, w, wx, rt, eb, smo);
    if constexpr (F >= 5) {
        // y again from its source (the object cache or global memory) through
        // the sorted index, rather than held in registers through phase B
        R yy[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const int j = t * PPL + p;
            yy[p] = j < n ? ysrc[(int)(G.SK[j] & 0xffffu)] : R(0);
        }
        return chi2_of<P, NW, PPL>(G, w, yy, smo);
    } else {
        return chi2_of<P, NW, PPL>(G, w, y, smo);
    }
}

// ------------------------------------------------------------------ Sec. 3
// One sweep over the candidate spans (smooths s_k, traces TR_k).  First
// reading (GV = false): generalized cross-validation picks one span per
// trial, chi^2 = RSS of that span.  Second reading (GV = true): a span per
// point by the un-smoothed generalized-validation residual
// |y - s_k| / (1 - TR_k/n), Listing 1's scan, bass enhancement, clip and
// blend of the s_k, chi^2 of the blend (no residual, span or final smooth).
template <class P, int NW, int PPL, bool GV, int F>
__device__ double single_pass(const Group<P, NW, PPL, F> &G, const TrialLaunch &L,
                              const typename P::S (&x)[PPL], const typename P::R (&w)[PPL],
                              const typename P::S (&wx)[PPL], const typename P::R (&y)[PPL]) {
    using R = typename P::R;
    using Geo = typename P::Geo;
    const int n = G.n, t = G.t;
    const int K = L.fixed_span > 0.0 ? 1 : 3;
    int b[3];
    for (int k = 0; k < 3; ++k) b[k] = K == 1 ? G.hwf : G.hw[k];
    int e = b[0];
    for (int k = 1; k < K; ++k) e = b[k] > e ? b[k] : e;
    // A1: geometry of every candidate span, and the smoother traces
    Geo g[3][PPL];
    typename P::S tr[3] = {P::zero(), P::zero(), P::zero()};
    prefix_x<P, NW, PPL>(G, x, w, wx, e);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = min(t * PPL + p, n - 1);
        const R wk = t * PPL + p < n ? w[p] : R(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k < K) {
                R h;
                g[k][p] = geometry<P, NW, PPL>(G, j, b[k], x[p], h);
                tr[k] = P::add(tr[k], P::prod(wk, h));
            }
        }
    }
    // A2: one prefix of y, every candidate smooth
    R s[3][PPL];
    prefix_pair<P, NW, PPL>(G, w, wx, y, e);
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = min(t * PPL + p, n - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) s[k][p] = k < K ? window_fit<P, NW, PPL>(G, g[k][p], j, b[k]) : R(0);
    }
    if (G.ties) {
#pragma unroll
        for (int k = 0; k < 3; ++k)
            if (k < K) tie_average<P, NW, PPL>(G, w, s[k]);
    }
    if constexpr (GV) {
        if (K == 3) {
            double trd[3] = {P::dbl(tr[0]), P::dbl(tr[1]), P::dbl(tr[2])};
            group_sum2<P, NW, PPL>(G, trd[0], trd[1]);
            trd[2] = group_sum1<P, NW, PPL>(G, trd[2]);
            bool ok[3];
            R iden[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double den = 1.0 - trd[k] * G.inv_n;  // > 0 whenever TR_k < n
                ok[k] = trd[k] < (double)n && den > 0.0;
                iden[k] = ok[k] ? (R)rcp64(den) : R(0);
            }
            const R sp0 = (R)L.span[0], sp1 = (R)L.span[1], sp2 = (R)L.span[2];
            const R spk[3] = {sp0, sp1, sp2};
            const R ilo = G.ilo, ihi = G.ihi;
            const double alpha = L.alpha;
            const bool bass = alpha > 0.0 && alpha <= 10.0;
            const R ex = (R)(10.0 - alpha);
            // spans with the same half-width give the same smooth: reuse the
            // residual so that the scan's tie rule (first span wins) sees an
            // exact tie, as the definition does
            const bool same01 = b[1] == b[0], same12 = b[2] == b[1];
            R smo[PPL];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                R e[3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    e[k] = ok[k] ? P::fabs_(y[p] - s[k][p]) * iden[k] : R(__builtin_inff());
                if (same01) e[1] = e[0];
                if (same12) e[2] = e[1];
                R resmin = R(1.0e20), sel = R(0);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    const bool lt = e[k] < resmin;
                    resmin = lt ? e[k] : resmin;
                    sel = lt ? spk[k] : sel;
                }
                if (bass && resmin < e[2] && resmin > R(0)) {
                    R tmp = resmin / e[2];
                    if (tmp < R(1.0e-7)) tmp = R(1.0e-7);
                    sel += (sp2 - sel) * bass_pow<P>(tmp, ex);
                }
                if (sel <= sp0) sel = sp0;
                if (sel >= sp2) sel = sp2;
                const R f = sel - sp1;
                const bool below = f < R(0);
                const R fr = below ? f * ilo : f * ihi;
                smo[p] = (R(1) - fr) * s[1][p] + fr * (below ? s[0][p] : s[2][p]);
            }
            return chi2_of<P, NW, PPL>(G, w, y, smo);
        }
    }
    double best = 0.0, chi2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k >= K) break;
        auto rss = P::zero();
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            const R d = t * PPL + p < n ? y[p] - s[k][p] : R(0);
            rss = P::add(rss, P::prod(w[p] * d, d));
        }
        double rss_d = P::dbl(rss), tr_d = P::dbl(tr[k]);
        group_sum2<P, NW, PPL>(G, rss_d, tr_d);
        double gcv = __builtin_inf();
        const double den = 1.0 - tr_d * G.inv_n;
        if (tr_d < (double)n && den * den > 0.0) gcv = rss_d * rcp64(den * den);
        if (k == 0 || gcv < best) {
            best = gcv;
            chi2 = rss_d;
        }
    }
    return chi2;
}

// ------------------------------------------------------------------ phase dispersion
// Number of sorted points whose 48-bit phase is below `bnd`.
__device__ __forceinline__ int count_below(const uint64_t *SK, int n, uint64_t bnd) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((SK[mid] >> 16) < bnd)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

// A second finder on the same fold and sort: the fraction of chi0 explained
// by the weighted means of B equal phase bins.  Bin b holds the sorted points
// with b 2^48 <= B phase48 < (b + 1) 2^48, a contiguous run found by binary
// search on the sorted keys; its sums are differences of prefix sums of w and
// w y built in A0, A1 (free until the smoother starts).
template <class P, int NW, int PPL, int F>
__device__ double pdm_score(const Group<P, NW, PPL, F> &G, int B, const typename P::R (&w)[PPL],
                            const typename P::R (&y)[PPL], double chi0) {
    using S = typename P::S;
    S q[2][PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        q[0][p] = P::from(w[p]);
        q[1][p] = P::prod(w[p], y[p]);
    }
    S *const Pf[2] = {G.Q, G.Q + 1};
    S T[2];
    bsync<NW>();
    build_prefix<P, NW, PPL, 2, false>(G, Pf, q, T);
    const int n = G.n;
    const uint64_t one = 1ull << 48;
    double e = 0.0;
    for (int b = G.t; b < B; b += Group<P, NW, PPL, F>::NT) {
        const int lo = count_below(G.SK, n, ((uint64_t)b * one + (uint64_t)(B - 1)) / (uint64_t)B);
        const int hi = b == B - 1 ? n
                                  : count_below(G.SK, n,
                                                ((uint64_t)(b + 1) * one + (uint64_t)(B - 1)) /
                                                    (uint64_t)B);
        const double wb = P::dbl(P::sub(G.Q[G.at(hi)], G.Q[G.at(lo)]));
        const double sb = P::dbl(P::sub(G.Q[G.at(hi) + 1], G.Q[G.at(lo) + 1]));
        if (wb > 0.0) e += sb * sb / wb;
    }
    return group_sum1<P, NW, PPL>(G, e) / chi0;
}

// ------------------------------------------------------------------ one trial
// Object data of the work item, original (time) order; re-read from the
// caches at every trial instead of being held in registers.
template <class P>
struct ObjData {
    const double *tt;
    const typename P::R *y, *w;
};

// Fold (FP64) and stable sort of one trial frequency: the sorted keys in SK
// (48-bit phase, point index in the low 16 bits), G.ties, G.vsmlsq.  Needs
// only the times, so objects that share them share this step.  Returns true
// when the sorted phases do not spread (Listing 1's constant fit).
// Phase key of point j with time x at frequency f: the 48-bit fixed-point
// phase in the high bits, j in the low 16 (stable order on equal phases);
// all ones for padding slots (j >= n).
__device__ __forceinline__ uint64_t phase_key(double x, double f, int j, int n) {
    // fraction of the exact product tt f (one rounding, the same for every
    // point); clamped at 0 where tt f lies just below an integer that its
    // rounded value reached, so that ph is always in [0, 1)
    const double ph = fmax(fma(x, f, -floor(x * f)), 0.0);
    // floor(ph 2^48), an integer below 2^48: adding 2^52 places it exactly
    // in the low mantissa bits (cheaper than a general double -> uint64)
    const double q = floor(ph * 0x1p48) + 0x1p52;
    const uint64_t ph48 = __builtin_bit_cast(uint64_t, q) & ((1ull << 52) - 1);
    return j < n ? ((ph48 << 16) | (uint64_t)j) : ~0ull;
}

// Flat-phase test and the smallest-variance threshold from the sorted keys
// (shared by both sorts).
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ bool sorted_scale(Group<P, NW, PPL, F> &G, const uint64_t *SK) {
    const int n = G.n;
    if ((SK[n - 1] >> 16) <= (SK[0] >> 16)) return true;
    const int q = n / 4;
    const double scale =
        (double)(SK[3 * q - 1] >> 16) * 0x1p-48 - (double)(SK[q - 1] >> 16) * 0x1p-48;
    G.vsmlsq = listing_vsmlsq(scale);
    return false;
}

template <class P, int NW, int PPL, bool CACHE_TT, int F>
__device__ bool fold_sort(Group<P, NW, PPL, F> &G, unsigned char *lds, const Layout &Y,
                          const double *tt_global, double f) {
    const int n = G.n, t = G.t, NP = Y.np;
    const double *ct = (const double *)(lds + Y.obj);  // cached times (CACHE_TT)
    // ---- fold (FP64): phase = frac(tt*f), as a 48-bit fixed-point key with
    // the point index in the low 16 bits (stable order on equal phases)
    uint64_t key[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = t * PPL + p;
        key[p] = phase_key((CACHE_TT ? ct : tt_global)[min(j, n - 1)], f, j, n);
    }
    // ---- bucket sort in LDS: NP buckets on the top phase bits, counts by LDS
    // atomics, a group scan for the bucket starts, then the exact rank inside
    // a bucket by comparing against its (few) members.  The counters are
    // zero on entry (cleared at the end of the previous sort, behind at least
    // one group barrier); the bucketed keys go to the prefix region, which
    // is dead until the smoother starts and is first written after two
    // barriers here.
    uint32_t *cnt = (uint32_t *)(lds + Y.cnt);
    uint64_t *tmp = (uint64_t *)lds;
    uint64_t *SK = (uint64_t *)(lds + Y.sk);
    int bkt[PPL];
    uint32_t slot[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = t * PPL + p;
        bkt[p] = (int)(((key[p] >> 32) * (uint64_t)NP) >> 32);
        slot[p] = 0u;
        if (j < n) slot[p] = atomicAdd(&cnt[bkt[p]], 1u);
    }
    bsync<NW>();
    {
        uint32_t c[PPL], tot = 0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            c[p] = cnt[t * PPL + p];
            tot += c[p];
        }
        const uint32_t incl = wave_incl_sum_u32(tot);
        uint32_t run = incl - tot;
        if constexpr (NW > 1) {
            uint32_t *xu = (uint32_t *)G.xd;
            if (G.lane == kWave - 1) xu[G.wave] = incl;
            __syncthreads();
            for (int w = 0; w < G.wave; ++w) run += xu[w];
        }
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            cnt[t * PPL + p] = run;
            run += c[p];
        }
        if (t == Group<P, NW, PPL, F>::NT - 1) cnt[NP] = run;
    }
    bsync<NW>();
    // bucket bounds [bs, be) of every slot, read once for the scatter and the
    // ranking (the counters hold the bucket starts until the end of the sort)
    uint32_t bs[PPL], be[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        bs[p] = cnt[bkt[p]];
        be[p] = cnt[bkt[p] + 1];
    }
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = t * PPL + p;
        if (j < n) tmp[bs[p] + slot[p]] = key[p];
    }
    bsync<NW>();
    // rank inside the bucket; equal phases share a bucket, so a tie is two
    // members of one bucket with the same phase.  The first kRankU members of
    // every slot's bucket are loaded together (one LDS round trip for all
    // slots rather than one per member); only longer buckets loop.  Loads
    // past a bucket's end are not used.
    bool tie = false;
    uint64_t mem[PPL][kRankU];
#pragma unroll
    for (int p = 0; p < PPL; ++p)
#pragma unroll
        for (int u = 0; u < kRankU; ++u) mem[p][u] = tmp[bs[p] + u];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = t * PPL + p;
        if (j < n) {
            const uint32_t s = bs[p], e = be[p];
            const uint64_t ph = key[p] >> 16;
            uint32_t rank = 0;
#pragma unroll
            for (int u = 0; u < kRankU; ++u) {
                const uint64_t o = mem[p][u];
                const bool in = s + u < e;
                rank += (in && o < key[p]) ? 1u : 0u;
                tie |= in && (o >> 16) == ph && o != key[p];
            }
            for (uint32_t i = s + kRankU; i < e; ++i) {
                const uint64_t o = tmp[i];
                rank += o < key[p] ? 1u : 0u;
                tie |= (o >> 16) == ph && o != key[p];
            }
            SK[s + rank] = key[p];
        }
    }
    if constexpr (NW == 1) {
        wave_lds_sync();
        G.ties = wave_ballot(tie) != 0;
    } else {
        G.ties = __syncthreads_or(tie) != 0;
    }
    // every rank is taken: clear the counters for the next sort
#pragma unroll
    for (int p = 0; p < PPL; ++p) cnt[t * PPL + p] = 0u;
    return sorted_scale(G, SK);
}

// The smoother and the score of one object on the sorted keys of fold_sort:
// gathers the object's y, w in phase order (from the item's LDS object cache,
// or from global memory through the key's index), runs Listing 1 or the
// single-pass variant, returns P = 1 - chi2/chi0.
template <class P, int NW, int PPL, int METHOD, bool PDM, bool CACHE_YW, int F>
__device__ double score_sorted(Group<P, NW, PPL, F> &G, unsigned char *lds, const Layout &Y,
                               const TrialLaunch &L, const typename P::R *y_src,
                               const typename P::R *w_src, bool flat, double chi0, double &pdm) {
    using R = typename P::R;
    using S = typename P::S;
    const int n = G.n, t = G.t, NP = Y.np;
    const R *cy = (const R *)(lds + Y.obj + NP * 8);
    const R *cw = (const R *)(lds + Y.obj + 2 * NP * 8);
    const uint64_t *SK = (const uint64_t *)(lds + Y.sk);
    S x[PPL], wx[PPL];
    R y[PPL], w[PPL];
#pragma unroll
    for (int p = 0; p < PPL; ++p) {
        const int j = t * PPL + p;
        const bool ok = j < n;
        const uint64_t k = ok ? SK[j] : ~0ull;
        const int i = ok ? (int)(k & 0xffffu) : 0;  // original index of the sorted point
        y[p] = ok ? (CACHE_YW ? cy : y_src)[i] : R(0);
        w[p] = ok ? (CACHE_YW ? cw : w_src)[i] : R(0);
        x[p] = ok ? P::x_of_key(k) : P::zero();
        wx[p] = P::mulr(x[p], w[p]);
    }
    if constexpr (PDM) {
        const int B = L.pdm_bins > 0 ? L.pdm_bins : min(32, max(4, n / 5));
        pdm = pdm_score<P, NW, PPL>(G, B, w, y, chi0);
    }
    // ---- Listing 1: constant fit when the phases do not spread
    if (flat) {
        double a = 0.0, sw_ = 0.0;
#pragma unroll
        for (int p = 0; p < PPL; ++p) {
            a += (double)w[p] * (double)y[p];
            sw_ += (double)w[p];
        }
        group_sum2<P, NW, PPL>(G, a, sw_);
        const R m = (R)(sw_ > 0.0 ? a / sw_ : 0.0);
        R smo[PPL];
#pragma unroll
        for (int p = 0; p < PPL; ++p) smo[p] = m;
        return 1.0 - chi2_of<P, NW, PPL>(G, w, y, smo) * G.inv_chi0;
    }
    const double chi2 = (METHOD == 0) ? supersmoother<P, NW, PPL>(G, L, x, w, wx, y,
                                                                  CACHE_YW ? cy : y_src)
                                      : single_pass<P, NW, PPL, METHOD == 2>(G, L, x, w, wx, y);
    return 1.0 - chi2 * G.inv_chi0;
}

// Objects longer than the object cache (groups of more than 1,024 points)
// read y, w from global memory through the sorted index.
template <class P, int NW, int PPL, int METHOD, bool PDM, int F>
__device__ double run_trial(Group<P, NW, PPL, F> &G, unsigned char *lds, const Layout &Y,
                            const TrialLaunch &L, const ObjData<P> &od, double f, double chi0,
                            double &pdm) {
    constexpr bool kCache = caches_object(kWave * NW * PPL);
    const bool flat = fold_sort<P, NW, PPL, kCache>(G, lds, Y, od.tt, f);
    return score_sorted<P, NW, PPL, METHOD, PDM, kCache>(G, lds, Y, L, od.y, od.w, flat, chi0,
                                                         pdm);
}

// Per-length values of a work item, once per item (the trials multiply by
// 1/n; the half-widths are taken here rather than per trial).
template <class P, int NW, int PPL, int F>
__device__ __forceinline__ void set_length(Group<P, NW, PPL, F> &G, const TrialLaunch &L, int n) {
    G.n = n;
    G.inv_n = 1.0 / (double)n;
    for (int k = 0; k < 3; ++k) G.hw[k] = halfwidth(n, L.span[k]);
    G.hwf = L.fixed_span > 0.0 ? halfwidth(n, L.fixed_span) : 0;
}

// One work item: an object and a run of consecutive trial frequencies (a tile
// of the full grid, or one refine range).
template <class P, int NW, int PPL, int METHOD, bool PDM, int F>
__device__ void run_item(Group<P, NW, PPL, F> &G, unsigned char *lds, const Layout &Y,
                         const TrialLaunch &L, int64_t item) {
    using R = typename P::R;
    const int64_t ci = item / L.n_tiles;
    const int32_t tile = (int32_t)(item - ci * L.n_tiles);
    const int obj = uniform_i32(L.objs[ci]);
    const int64_t part = (int64_t)obj * L.n_tiles + tile;
    int64_t k0, k1;
    if (L.ranges) {
        k0 = uniform_i64(L.ranges[2 * part]);
        k1 = uniform_i64(L.ranges[2 * part + 1]);
    } else {
        k0 = (int64_t)tile * L.tile_f;
        k1 = (k0 + L.tile_f < L.n_freq) ? k0 + L.tile_f : L.n_freq;
    }
    const int64_t row = (int64_t)obj * L.n_freq;

    if (L.cat.status[obj] != 0) {
        for (int64_t k = k0 + G.t; k < k1; k += kWave * NW) {
            if (L.pgram64) L.pgram64[row + k] = __builtin_nan("");
            if (L.pgram32) L.pgram32[row + k] = __builtin_nanf("");
            if (L.pdm64) L.pdm64[row + k] = __builtin_nan("");
            if (L.pdm32) L.pdm32[row + k] = __builtin_nanf("");
        }
        if (G.t == 0 && L.part_p) {
            L.part_p[part] = __builtin_nan("");
            L.part_k[part] = -1;
        }
        return;
    }
    const int64_t base = uniform_i64(L.cat.offsets[obj]);
    set_length(G, L, (int)(uniform_i64(L.cat.offsets[obj + 1]) - base));
    ObjData<P> od;
    od.tt = uniform_ptr(L.cat.tt + base);
    od.y = uniform_ptr((P::kIsF64 ? (const R *)L.cat.yc : (const R *)L.cat.yc32) + base);
    od.w = uniform_ptr((P::kIsF64 ? (const R *)L.cat.w : (const R *)L.cat.w32) + base);
    const double chi0 = L.cat.chi0[obj];
    G.inv_chi0 = 1.0 / chi0;
    if constexpr (caches_object(kWave * NW * PPL)) {
        double *ct = (double *)(lds + Y.obj);
        R *cy = (R *)(lds + Y.obj + Y.np * 8);
        R *cw = (R *)(lds + Y.obj + 2 * Y.np * 8);
        for (int i = G.t; i < G.n; i += kWave * NW) {
            ct[i] = od.tt[i];
            cy[i] = od.y[i];
            cw[i] = od.w[i];
        }
        bsync<NW>();
    }
    double best_p = 0.0;
    int32_t best_k = -1;
    for (int64_t k = k0; k < k1; ++k) {
        const double f = grid_freq(L.fmin, L.df, k);
        double pdm = 0.0;
        const double Pk = run_trial<P, NW, PPL, METHOD, PDM>(G, lds, Y, L, od, f, chi0, pdm);
        if (G.t == 0) {
            if (L.pgram64) L.pgram64[row + k] = Pk;
            if (L.pgram32) L.pgram32[row + k] = (float)Pk;
            if (L.pdm64) L.pdm64[row + k] = pdm;
            if (L.pdm32) L.pdm32[row + k] = (float)pdm;
        }
        if (!__builtin_isnan(Pk) && (best_k < 0 || Pk > best_p)) {
            best_p = Pk;
            best_k = (int32_t)k;
        }
    }
    if (G.t == 0 && L.part_p) {
        L.part_p[part] = best_k < 0 ? __builtin_nan("") : best_p;
        L.part_k[part] = best_k;
    }
}

// Shared time sampling (Sec. 2.2: objects observed at the same times fold
// and sort alike): a work item is a batch of up to L.shared_batch objects of
// the class and a frequency tile.  Every trial frequency is folded and
// sorted once; each object of the batch then gathers its own y, w through
// the sorted index and runs the smoother.  The item's running maxima are
// kept in LDS (written by thread 0 only).
template <class P, int NW, int PPL, int METHOD, int F>
__device__ void run_item_shared(Group<P, NW, PPL, F> &G, unsigned char *lds, const Layout &Y,
                                const TrialLaunch &L, int64_t item) {
    using R = typename P::R;
    const int64_t bi = item / L.n_tiles;
    const int32_t tile = (int32_t)(item - bi * L.n_tiles);
    const int count = *L.count;
    const int m0 = (int)(bi * L.shared_batch);
    const int m1 = min(m0 + L.shared_batch, count);
    const int64_t k0 = (int64_t)tile * L.tile_f;
    const int64_t k1 = (k0 + L.tile_f < L.n_freq) ? k0 + L.tile_f : L.n_freq;
    double *bp = (double *)(lds + Y.best);
    int32_t *bk = (int32_t *)(lds + Y.best + kMaxSharedBatch * 8);
    // a batch without a usable object does no trial (its light curves may be
    // too short or too long for this group)
    bool any_ok = false;
    for (int m = m0; m < m1; ++m) any_ok |= L.cat.status[L.objs[m]] == 0;
    if (!any_ok) {
        for (int m = m0; m < m1; ++m) {
            const int64_t row = (int64_t)L.objs[m] * L.n_freq;
            for (int64_t k = k0 + G.t; k < k1; k += kWave * NW) {
                if (L.pgram64) L.pgram64[row + k] = __builtin_nan("");
                if (L.pgram32) L.pgram32[row + k] = __builtin_nanf("");
            }
            if (G.t == 0 && L.part_p) {
                const int64_t part = (int64_t)L.objs[m] * L.n_tiles + tile;
                L.part_p[part] = __builtin_nan("");
                L.part_k[part] = -1;
            }
        }
        return;
    }
    set_length(G, L, L.shared_n);
    constexpr bool kCache = caches_object(kWave * NW * PPL);
    if constexpr (kCache) {
        double *ct = (double *)(lds + Y.obj);
        for (int i = G.t; i < G.n; i += kWave * NW) ct[i] = L.shared_tt[i];
    }
    if (G.t == 0)
        for (int m = 0; m < m1 - m0; ++m) {
            bp[m] = 0.0;
            bk[m] = -1;
        }
    bsync<NW>();
    for (int64_t k = k0; k < k1; ++k) {
        const double f = grid_freq(L.fmin, L.df, k);
        const bool flat = fold_sort<P, NW, PPL, kCache>(G, lds, Y, L.shared_tt, f);
        for (int m = m0; m < m1; ++m) {
            const int obj = uniform_i32(L.objs[m]);
            const int64_t row = (int64_t)obj * L.n_freq;
            double Pk = __builtin_nan("");
            if (L.cat.status[obj] == 0) {
                const int64_t base = uniform_i64(L.cat.offsets[obj]);
                const double chi0 = L.cat.chi0[obj];
                G.inv_chi0 = 1.0 / chi0;
                const R *yo = (P::kIsF64 ? (const R *)L.cat.yc : (const R *)L.cat.yc32) + base;
                const R *wo = (P::kIsF64 ? (const R *)L.cat.w : (const R *)L.cat.w32) + base;
                double pdm = 0.0;
                Pk = score_sorted<P, NW, PPL, METHOD, false, false>(G, lds, Y, L, yo, wo, flat,
                                                                    chi0, pdm);
            }
            if (G.t == 0) {
                if (L.pgram64) L.pgram64[row + k] = Pk;
                if (L.pgram32) L.pgram32[row + k] = (float)Pk;
                const int i = m - m0;
                if (!__builtin_isnan(Pk) && (bk[i] < 0 || Pk > bp[i])) {
                    bp[i] = Pk;
                    bk[i] = (int32_t)k;
                }
            }
        }
    }
    if (G.t == 0 && L.part_p)
        for (int m = m0; m < m1; ++m) {
            const int64_t part = (int64_t)L.objs[m] * L.n_tiles + tile;
            const int i = m - m0;
            L.part_p[part] = bk[i] < 0 ? __builtin_nan("") : bp[i];
            L.part_k[part] = bk[i];
        }
}

// Minimum wavefronts per SIMD the compiler must fit each kernel into (its
// register budget: 512 / waves registers per lane).  Measured on MI355X per
// precision, shape and method: a budget that forces a few spills but raises
// the resident wavefronts pays off for some kernels (up to 1.8x) and costs
// others (the single-wavefront SS kernel at 4 points per thread loses 40 %
// when held to two), so every kernel has its own value; 1 = no bound.
template <bool F64, int NW, int PPL, int METHOD>
constexpr int waves_per_simd() {
    constexpr bool ss = METHOD == 0;
    if (NW == 1 && PPL == 1) return F64 ? (ss ? 4 : 1) : 1;
    if (NW == 1 && PPL == 2) return ss ? 1 : 3;
    if (NW == 1 && PPL == 3) return (F64 && ss) ? 2 : 1;
    if (NW == 1 && PPL == 4) return ss ? 1 : 2;
    if (NW == 2 && PPL == 1) return F64 ? 4 : (ss ? 3 : 1);
    if (NW == 2 && PPL == 2) return ss ? (F64 ? 3 : 1) : 3;
    if (NW == 4 && PPL == 1) return F64 ? 4 : (ss ? 3 : 1);
    if (NW == 2 && PPL == 3) return 1;  // FP64 SS held to 2 spilled to scratch and miscomputed
    if (NW == 2 && PPL == 4) return 1;  // FP64 SS miscomputed in an earlier build
    if (NW == 4 && PPL == 2) return ss ? (F64 ? 2 : 1) : 3;
    if (NW == 4 && PPL == 4) return ss ? 1 : 2;
    return 1;
}

// Persistent: every workgroup takes items from the class's queues until all
// count * n_tiles items are handed out (each workgroup exits after one failed
// take per queue).
template <class P, int NW, int PPL, int METHOD, bool PDM, bool SHARED = false>
__global__ __launch_bounds__(kWave *NW,
                             (PDM ? 1 : waves_per_simd<P::kIsF64, NW, PPL, METHOD>()))
void trial_kernel(TrialLaunch L) {
    using S = typename P::S;
    extern __shared__ __align__(16) unsigned char lds[];
    const Layout Y(NW, PPL, L.ext, METHOD);
    Group<P, NW, PPL, prefix_arrays(METHOD, NW, PPL)> G;
    G.Q = (S *)lds;
    G.SK = (const uint64_t *)(lds + Y.sk);
    G.xs = (S *)(lds + Y.xch);
    G.xd = (double *)(lds + Y.xch);
    G.t = threadIdx.x;
    G.wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // uniform per wavefront
    G.lane = threadIdx.x % kWave;
    G.ext = Y.ext;
    G.ties = false;
    G.vsmlsq = 0.0;
    G.inv_n = 0.0;
    G.inv_chi0 = 0.0;
    G.n = 0;
    for (int k = 0; k < 3; ++k) G.hw[k] = 0;
    G.hwf = 0;
    {  // once per kernel (a select between the two products was otherwise
       // turned into a division per point)
        using R = typename P::R;
        const R sp0 = (R)L.span[0], sp1 = (R)L.span[1], sp2 = (R)L.span[2];
        G.ilo = R(1) / (sp0 - sp1);
        G.ihi = R(1) / (sp2 - sp1);
    }
    {  // the sort's bucket counters start at zero (and every sort leaves them so)
        uint32_t *cnt = (uint32_t *)(lds + Y.cnt);
        for (int i = G.t; i < Y.np; i += kWave * NW) cnt[i] = 0u;
    }
    // units: the class's objects (or batches of objects sharing their times);
    // queue q hands out the (unit, tile) items of the units with u mod
    // kQueuesPerClass == q, all tiles of a unit in a row.  A workgroup starts
    // on the queue of its XCD and moves on to the next when one is empty, so
    // every workgroup exits after one failed take per queue.
    const unsigned long long units =
        SHARED ? (unsigned long long)((*L.count + L.shared_batch - 1) / L.shared_batch)
               : (unsigned long long)(*L.count);
    const unsigned long long n_tiles = (unsigned long long)L.n_tiles;
    unsigned long long *take = (unsigned long long *)(lds + Y.qslot);
    const int own = (int)(blockIdx.x % kQueuesPerClass);
    for (int k = 0; k < kQueuesPerClass; ++k) {
        const int q = (own + k) % kQueuesPerClass;
        const unsigned long long uq =
            units > (unsigned long long)q
                ? (units - q + kQueuesPerClass - 1) / kQueuesPerClass
                : 0ull;
        const unsigned long long total = uq * n_tiles;
        if (total == 0) continue;  // an empty queue needs no take
        for (;;) {
            bsync<NW>();
            if (G.t == 0) *take = atomicAdd(L.queue + q, 1ull);
            bsync<NW>();
            const unsigned long long local = *take;
            if (local >= total) break;
            const unsigned long long unit = q + kQueuesPerClass * (local / n_tiles);
            const int64_t item = (int64_t)(unit * n_tiles + local % n_tiles);
            if constexpr (SHARED)
                run_item_shared<P, NW, PPL, METHOD>(G, lds, Y, L, item);
            else
                run_item<P, NW, PPL, METHOD, PDM>(G, lds, Y, L, item);
        }
    }
}

template <class P, int NW, int PPL, int METHOD, bool PDM, bool SHARED = false>
hipError_t launch_variant(const TrialLaunch &L, int64_t max_items, int n_cu, hipStream_t s) {
    const Layout Y(NW, PPL, L.ext, METHOD);
    const void *fn = (const void *)trial_kernel<P, NW, PPL, METHOD, PDM, SHARED>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, Y.bytes);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kWave * NW, (size_t)Y.bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    int64_t grid = (int64_t)per_cu * n_cu;
    if (grid > max_items) grid = max_items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((trial_kernel<P, NW, PPL, METHOD, PDM, SHARED>), dim3((unsigned)grid),
                       dim3(kWave * NW), (size_t)Y.bytes, s, L);
    return hipGetLastError();
}

// The phase-dispersion finder is its own kernel variant, so that the plain
// kernels keep their register allocation.
template <class P, int NW, int PPL, int METHOD>
hipError_t launch_one(const TrialLaunch &L, int64_t max_items, int n_cu, hipStream_t s) {
    if (L.shared_batch > 0) return launch_variant<P, NW, PPL, METHOD, false, true>(L, max_items, n_cu, s);
    return (L.pdm64 || L.pdm32) ? launch_variant<P, NW, PPL, METHOD, true>(L, max_items, n_cu, s)
                                : launch_variant<P, NW, PPL, METHOD, false>(L, max_items, n_cu, s);
}

template <class P, int NW, int PPL>
hipError_t launch_cls(const TrialLaunch &L, int64_t max_items, int n_cu, hipStream_t s) {
    switch (L.method) {
    case 0: return launch_one<P, NW, PPL, 0>(L, max_items, n_cu, s);
    case 1: return launch_one<P, NW, PPL, 1>(L, max_items, n_cu, s);
    case 2: return launch_one<P, NW, PPL, 2>(L, max_items, n_cu, s);
    }
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ invariant checks
// Debug mode: the sort and the window code of the trial kernels run again
// over the same work items (the FP64 policy, the single-pass layout), and
// three counters are added to: trials checked, adjacent sorted keys that do
// not increase (keys carry the point index, so they are unique and must
// increase strictly: phases ascending, equal phases in index order), and
// windows of a used span whose weight sum W is not positive.  selftest
// inverts the order test, so that every trial of two or more points counts
// (to show that a violation is reported).  Non-persistent: workgroups stride
// over the class's items.
template <int NW, int PPL>
__global__ __launch_bounds__(kWave *NW) void check_kernel(TrialLaunch L,
                                                        unsigned long long *counts,
                                                        int selftest) {
    using P = F64;
    constexpr int F = prefix_arrays(1, NW, PPL);
    extern __shared__ __align__(16) unsigned char lds[];
    const Layout Y(NW, PPL, L.ext, 1);
    Group<P, NW, PPL, F> G;
    G.Q = (double *)lds;
    G.SK = (const uint64_t *)(lds + Y.sk);
    G.xs = (double *)(lds + Y.xch);
    G.xd = (double *)(lds + Y.xch);
    G.t = threadIdx.x;
    G.wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    G.lane = threadIdx.x % kWave;
    G.ext = Y.ext;
    G.ties = false;
    G.vsmlsq = 0.0;
    G.inv_chi0 = 0.0;
    G.ilo = G.ihi = 0.0;
    G.n = 0;
    G.inv_n = 0.0;
    for (int k = 0; k < 3; ++k) G.hw[k] = 0;
    G.hwf = 0;
    uint32_t *cnt = (uint32_t *)(lds + Y.cnt);
    for (int i = G.t; i < Y.np; i += kWave * NW) cnt[i] = 0u;
    unsigned long long n_trials = 0, n_order = 0, n_weight = 0;
    const long long items = (long long)(*L.count) * L.n_tiles;
    for (long long item = blockIdx.x; item < items; item += gridDim.x) {
        const int64_t ci = item / L.n_tiles;
        const int32_t tile = (int32_t)(item - ci * L.n_tiles);
        const int obj = uniform_i32(L.objs[ci]);
        if (L.cat.status[obj] != 0) continue;
        const int64_t k0 = (int64_t)tile * L.tile_f;
        const int64_t k1 = (k0 + L.tile_f < L.n_freq) ? k0 + L.tile_f : L.n_freq;
        const int64_t base = uniform_i64(L.cat.offsets[obj]);
        bsync<NW>();
        set_length(G, L, (int)(uniform_i64(L.cat.offsets[obj + 1]) - base));
        const int n = G.n;
        // the object's times and weights: cached in LDS as the trial kernels
        // do for groups of up to 1,024 points, else read from global memory
        constexpr bool kCache = caches_object(kWave * NW * PPL);
        const double *ct = L.cat.tt + base, *cw = L.cat.w + base;
        if constexpr (kCache) {
            double *lt = (double *)(lds + Y.obj), *lw = (double *)(lds + Y.obj + 2 * Y.np * 8);
            for (int i = G.t; i < n; i += kWave * NW) {
                lt[i] = ct[i];
                lw[i] = cw[i];
            }
            ct = lt;
            cw = lw;
        }
        bsync<NW>();
        const int fixed = L.fixed_span > 0.0;
        const int e = fixed ? G.hwf : G.hw[2];
        for (int64_t k = k0; k < k1; ++k) {
            const double f = grid_freq(L.fmin, L.df, k);
            const bool flat = fold_sort<P, NW, PPL, kCache>(G, lds, Y, ct, f);
            if (G.t == 0) ++n_trials;
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const int j = G.t * PPL + p;
                if (j + 1 < n) {
                    const bool up = G.SK[j + 1] > G.SK[j];
                    n_order += (selftest ? up : !up) ? 1u : 0u;
                }
            }
            if (flat) continue;
            double x[PPL], w[PPL], wx[PPL];
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const int j = G.t * PPL + p;
                const uint64_t key = j < n ? G.SK[j] : 0ull;
                w[p] = j < n ? cw[(int)(key & 0xffffu)] : 0.0;
                x[p] = j < n ? P::x_of_key(key) : 0.0;
                wx[p] = x[p] * w[p];
            }
            prefix_x<P, NW, PPL>(G, x, w, wx, e);
#pragma unroll
            for (int p = 0; p < PPL; ++p) {
                const int j = G.t * PPL + p;
                if (j >= n) continue;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    if (fixed ? s != 3 : s == 3) continue;
                    const int b = s == 3 ? G.hwf : G.hw[s];
                    const double W = G.Q[G.at(j + b + 1)] - G.Q[G.at(j - b)];
                    n_weight += W > 0.0 ? 0u : 1u;
                }
            }
        }
    }
    if (n_trials) atomicAdd(counts, n_trials);
    if (n_order) atomicAdd(counts + 1, n_order);
    if (n_weight) atomicAdd(counts + 2, n_weight);
}

template <int NW, int PPL>
hipError_t launch_check(const TrialLaunch &L, int64_t max_items, int n_cu,
                        unsigned long long *counts, int selftest, hipStream_t s) {
    const Layout Y(NW, PPL, L.ext, 1);
    const void *fn = (const void *)check_kernel<NW, PPL>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, Y.bytes);
    if (e != hipSuccess) return e;
    int64_t grid = (int64_t)4 * n_cu;
    if (grid > max_items) grid = max_items;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL((check_kernel<NW, PPL>), dim3((unsigned)grid), dim3(kWave * NW),
                       (size_t)Y.bytes, s, L, counts, selftest);
    return hipGetLastError();
}

hipError_t launch_checks_shape(int shape, const TrialLaunch &L, int64_t max_items, int n_cu,
                               unsigned long long *counts, int selftest, hipStream_t s) {
    switch (shape) {
#define SSG_CHECK_CASE(nw, ppl) \
    case shape_id(nw, ppl): return launch_check<nw, ppl>(L, max_items, n_cu, counts, selftest, s);
        SSG_SHAPES(SSG_CHECK_CASE)
#undef SSG_CHECK_CASE
    }
    return hipErrorInvalidValue;
}

template <class P>
hipError_t launch_policy(int shape, const TrialLaunch &L, int64_t max_items, int n_cu,
                         hipStream_t s) {
    switch (shape) {
#define SSG_SHAPE_CASE(nw, ppl) \
    case shape_id(nw, ppl): return launch_cls<P, nw, ppl>(L, max_items, n_cu, s);
        SSG_SHAPES(SSG_SHAPE_CASE)
#undef SSG_SHAPE_CASE
    }
    return hipErrorInvalidValue;
}

}  // namespace
}  // namespace ssg
