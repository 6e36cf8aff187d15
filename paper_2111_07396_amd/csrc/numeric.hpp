// Arithmetic policies of the trial kernel.
//
//   F64  : every per-point value and every prefix/window sum in FP64.
//   F32C : per-point values in FP32; prefix and window sums as unevaluated
//          float pairs (hi + lo, error-free transformations: Knuth's TwoSum,
//          Dekker's Fast2Sum, FMA-based TwoProduct), i.e. compensated FP32
//          summation carried through the parallel scan.  The phase keeps 48
//          bits as an exact float pair.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "wave.hpp"

namespace ssg {

// 1/a for FP64: the hardware estimate (about 2^-23 relative on gfx950) refined
// by one Newton step, r' = r + r (1 - a r), which squares the relative error:
// measured on 4M log-uniform values over 2^-30..2^30, at most 11 ulp from the
// correctly rounded quotient (a second step makes it exact there, for 2 more
// FMA per reciprocal; 11 ulp is far below the window sums' own rounding).
__device__ __forceinline__ double rcp64(double a) {
    const double r = __builtin_amdgcn_rcp(a);
    const double e = fma(-a, r, 1.0);
    return fma(e, r, r);
}



// ------------------------------------------------------------------ float pairs
struct df {
    float hi, lo;
};

__device__ __forceinline__ df two_sum(float a, float b) {
#pragma clang fp contract(off)
    float s = a + b;
    float bb = s - a;
    float e = (a - (s - bb)) + (b - bb);
    return {s, e};
}

__device__ __forceinline__ df fast_two_sum(float a, float b) {  // needs |a| >= |b| or a == 0
#pragma clang fp contract(off)
    float s = a + b;
    float e = b - (s - a);
    return {s, e};
}

__device__ __forceinline__ df two_prod(float a, float b) {
#pragma clang fp contract(off)
    float p = a * b;
    float e = __builtin_fmaf(a, b, -p);
    return {p, e};
}

// Pair sum with error about 2^-48 (|a| + |b|): enough for window sums taken
// as differences of prefix sums.
__device__ __forceinline__ df df_add(df a, df b) {
#pragma clang fp contract(off)
    df s = two_sum(a.hi, b.hi);
    float e = s.lo + (a.lo + b.lo);
    return fast_two_sum(s.hi, e);
}

__device__ __forceinline__ df df_neg(df a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ df df_sub(df a, df b) { return df_add(a, df_neg(b)); }

__device__ __forceinline__ df df_mul(df a, df b) {
#pragma clang fp contract(off)
    df p = two_prod(a.hi, b.hi);
    float e = __builtin_fmaf(a.hi, b.lo, p.lo);
    e = __builtin_fmaf(a.lo, b.hi, e);
    return fast_two_sum(p.hi, e);
}

__device__ __forceinline__ df df_mul_f(df a, float b) {
#pragma clang fp contract(off)
    df p = two_prod(a.hi, b);
    float e = __builtin_fmaf(a.lo, b, p.lo);
    return fast_two_sum(p.hi, e);
}

__device__ __forceinline__ df readlane_df(df v, int lane) {
    return {readlane_f32(v.hi, lane), readlane_f32(v.lo, lane)};
}

template <int CTRL, int ROWMASK, bool BC>
__device__ __forceinline__ df dpp_df(df v) {
    return {dpp_f32<CTRL, ROWMASK, BC>(v.hi), dpp_f32<CTRL, ROWMASK, BC>(v.lo)};
}

__device__ __forceinline__ df wave_incl_sum_df(df x) {
    x = df_add(x, dpp_df<0x111, 0xf, true>(x));
    x = df_add(x, dpp_df<0x112, 0xf, true>(x));
    x = df_add(x, dpp_df<0x114, 0xf, true>(x));
    x = df_add(x, dpp_df<0x118, 0xf, true>(x));
    x = df_add(x, dpp_df<0x142, 0xa, false>(x));
    x = df_add(x, dpp_df<0x143, 0xc, false>(x));
    return x;
}

// Cross-row scan temporaries of the FP64 policy (wave_incl_sum_z); the
// float-pair policy clears its own.
struct ScanZ64 {
    double z15 = 0.0, z31 = 0.0;
};
struct ScanZNone {};

// ------------------------------------------------------------------ policies
struct F64 {
    using R = double;  // per-point values
    using S = double;  // prefix / window sums and the phase
    static constexpr bool kIsF64 = true;
    __device__ static S add(S a, S b) { return a + b; }
    __device__ static S sub(S a, S b) { return a - b; }
    __device__ static S neg(S a) { return -a; }
    __device__ static S twice(S a) { return 2.0 * a; }
    __device__ static S scale(S a, R q) { return a * q; }  // exact for q in {-1, 0, 1, 2}
    __device__ static S mul(S a, S b) { return a * b; }
    __device__ static S mulr(S a, R b) { return a * b; }
    __device__ static S prod(R a, R b) { return a * b; }
    __device__ static S from(R a) { return a; }
    __device__ static R real(S a) { return a; }
    __device__ static double dbl(S a) { return a; }
    __device__ static S zero() { return 0.0; }
    __device__ static S quot(S a, S /*b*/, R ib) { return a * ib; }
    using Z = ScanZ64;
    __device__ static S scan(S x, Z &z) { return wave_incl_sum_z(x, z.z15, z.z31); }
    template <int M>
    __device__ static void scan_n(const S (&x)[M], S (&out)[M], Z &z) {
#pragma unroll
        for (int m = 0; m < M; ++m) out[m] = x[m];
        wave_incl_sum_z_multi<M>(out, z.z15, z.z31);
    }
    __device__ static S lane_value(S x, int lane) { return readlane_f64(x, lane); }
    __device__ static R rcp(R a) { return rcp64(a); }
    __device__ static R fabs_(R a) { return fabs(a); }
    __device__ static S x_of_key(uint64_t key) { return (double)(key >> 16) * 0x1p-48; }
    __device__ static R exp2_log2_pow(R t, R e) {
        return (double)__builtin_amdgcn_exp2f((float)e * __builtin_amdgcn_logf((float)t));
    }
    // Window geometry: the local line through a window evaluated at x_j is
    // linear in the window sums of w v and w x v: s = A Sv + B Sxv with
    // B = (x_j - xm)/V (0 when V <= vsmlsq) and A = 1/W - xm B.  h is the
    // leverage term 1/W + (x_j - xm)^2/V.
    struct Geo {
        double A, B;
    };
    __device__ static Geo geo(S W, S Sx, S Sxx, S xj, double vsmlsq, R &h) {
        const double iW = rcp64(W);
        const double xm = Sx * iW;
        const double V = Sxx - Sx * xm;
        const double iV = V > vsmlsq ? rcp64(V) : 0.0;
        const double dx = xj - xm;
        Geo g;
        g.B = iV * dx;
        g.A = iW - xm * g.B;
        h = iW + dx * g.B;
        return g;
    }
    __device__ static R eval(const Geo &g, S Sv, S Sxv) { return fma(g.A, Sv, g.B * Sxv); }
};

struct F32C {
    using R = float;
    using S = df;
    static constexpr bool kIsF64 = false;
    __device__ static S add(S a, S b) { return df_add(a, b); }
    __device__ static S sub(S a, S b) { return df_sub(a, b); }
    __device__ static S neg(S a) { return df_neg(a); }
    __device__ static S twice(S a) { return {2.0f * a.hi, 2.0f * a.lo}; }
    __device__ static S scale(S a, R q) { return {a.hi * q, a.lo * q}; }  // q in {-1, 0, 1, 2}
    __device__ static S mul(S a, S b) { return df_mul(a, b); }
    __device__ static S mulr(S a, R b) { return df_mul_f(a, b); }
    __device__ static S prod(R a, R b) { return two_prod(a, b); }
    __device__ static S from(R a) { return {a, 0.0f}; }
    __device__ static R real(S a) { return a.hi + a.lo; }
    __device__ static double dbl(S a) { return (double)a.hi + (double)a.lo; }
    __device__ static S zero() { return {0.0f, 0.0f}; }
    // a/b to pair precision from an estimate of 1/b
    __device__ static S quot(S a, S b, R ib) {
        float q1 = a.hi * ib;
        df r = df_sub(a, df_mul_f(b, q1));
        float q2 = r.hi * ib;
        return fast_two_sum(q1, q2);
    }
    using Z = ScanZNone;
    __device__ static S scan(S x, Z &) { return wave_incl_sum_df(x); }
    template <int M>
    __device__ static void scan_n(const S (&x)[M], S (&out)[M], Z &) {
#pragma unroll
        for (int m = 0; m < M; ++m) out[m] = wave_incl_sum_df(x[m]);
    }
    __device__ static S lane_value(S x, int lane) { return readlane_df(x, lane); }
    __device__ static R rcp(R a) { return __builtin_amdgcn_rcpf(a); }
    __device__ static R fabs_(R a) { return fabsf(a); }
    __device__ static S x_of_key(uint64_t key) {
        uint64_t ph = key >> 16;  // 48-bit phase: exactly hi (top 24 bits) + lo
        return fast_two_sum((float)(uint32_t)(ph >> 24) * 0x1p-24f,
                            (float)(uint32_t)(ph & 0xffffffu) * 0x1p-48f);
    }
    __device__ static R exp2_log2_pow(R t, R e) {
        return __builtin_amdgcn_exp2f(e * __builtin_amdgcn_logf(t));
    }
    // s = Sv/W + B (Sxv - xm Sv) with the covariance term formed in pair
    // precision (it cancels heavily when the window sits far from x = 0).
    struct Geo {
        float iW, B;
        df xm;
    };
    __device__ static Geo geo(S W, S Sx, S Sxx, S xj, double vsmlsq, R &h) {
        Geo g;
        g.iW = rcp(real(W));
        g.xm = quot(Sx, W, g.iW);
        const float V = real(df_sub(Sxx, df_mul(Sx, g.xm)));
        const float iV = (double)V > vsmlsq ? rcp(V) : 0.0f;
        const float dx = real(df_sub(xj, g.xm));
        g.B = iV * dx;
        h = g.iW + dx * g.B;
        return g;
    }
    __device__ static R eval(const Geo &g, S Sv, S Sxv) {
        return real(Sv) * g.iW + g.B * real(df_sub(Sxv, df_mul(g.xm, Sv)));
    }
};

}  // namespace ssg
