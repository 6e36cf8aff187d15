// Per-object preparation (Alg. 1, compute_chi0_tt_weights) and the final
// per-object argmax over tile partials (Alg. 1, findPeriod).
#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

constexpr int kPrepWaves = 4;

__device__ __forceinline__ int pick_shape(const ShapeRules &R, int64_t n) {
    for (int i = 0; i < R.n_rules; ++i)
        if (n <= R.rule_n[i]) return R.rule_shape[i];
    for (int i = 0; i < R.n_def; ++i)
        if (n <= R.def_n[i]) return R.def_shape[i];
    return -1;
}

__global__ void reset_kernel(int32_t *counts, unsigned long long *queues, int n) {
    const int i = threadIdx.x;
    if (i < n) counts[i] = 0;
    for (int q = i; q < n * kQueuesPerClass; q += blockDim.x) queues[q] = 0ull;
}

// One wavefront per object.  FP64 throughout.  Status precedence: fewer than
// 5 points, non-finite t or y, bad error bar, chi0 == 0, too long.  Lane 0
// then files the object in its shape class.
__global__ __launch_bounds__(kWave *kPrepWaves) void prep_kernel(
    const int64_t *__restrict__ offsets, const double *__restrict__ t,
    const double *__restrict__ y, const double *__restrict__ e, int64_t n_obj, int64_t n_points,
    double *__restrict__ tt, double *__restrict__ w, double *__restrict__ yc,
    float *__restrict__ w32, float *__restrict__ yc32, double *__restrict__ chi0,
    double *__restrict__ sw_out, int32_t *__restrict__ status, ShapeRules rules, int32_t *__restrict__ objs,
    int32_t *__restrict__ counts, int shared_t) {
    const int lane = threadIdx.x % kWave;
    const int64_t obj = (int64_t)blockIdx.x * kPrepWaves + threadIdx.x / kWave;
    if (obj >= n_obj) return;
    const int64_t a = offsets[obj], n = offsets[obj + 1] - a;
    int32_t st = 0;
    double c0 = __builtin_nan(""), swt = __builtin_nan("");
    if (a < 0 || n < 0 || a + n > n_points) {
        st = 6;
    } else if (n < 5) {
        st = 1;
    } else {
        bool nonfinite = false, baderr = false;
        double tmin = __builtin_inf(), sw = 0.0, swy = 0.0;
        for (int64_t i = lane; i < n; i += kWave) {
            const double ti = t[shared_t ? i : a + i], yi = y[a + i], ei = e[a + i];
            nonfinite |= !__builtin_isfinite(ti) || !__builtin_isfinite(yi);
            baderr |= !__builtin_isfinite(ei) || !(ei > 0.0);
            tmin = fmin(tmin, ti);
            const double wi = 1.0 / (ei * ei);
            sw += wi;
            swy += wi * yi;
        }
        nonfinite = wave_ballot(nonfinite) != 0;
        baderr = wave_ballot(baderr) != 0;
        st = nonfinite ? 3 : (baderr ? 2 : 0);
        if (st == 0) {
            tmin = wave_min(tmin);
            sw = wave_sum(sw);
            swy = wave_sum(swy);
            swt = sw;
            const double ybar = swy / sw;
            double acc = 0.0;
            for (int64_t i = lane; i < n; i += kWave) {
                const double ei = e[a + i];
                const double wi = 1.0 / (ei * ei);
                const double d = y[a + i] - ybar;
                acc += wi * d * d;
                tt[a + i] = t[shared_t ? i : a + i] - tmin;
                w[a + i] = wi;
                yc[a + i] = d;
                w32[a + i] = (float)wi;
                yc32[a + i] = (float)d;
            }
            c0 = wave_sum(acc);
            if (!(c0 > 0.0)) st = 4;
        }
    }
    if (lane == 0) {
        int cls = (st != 6 && n >= 1) ? pick_shape(rules, n) : rules.fallback;
        if (st != 6 && (n > rules.max_points || cls < 0 || !((rules.runnable >> cls) & 1u))) {
            if (st == 0) st = 5;
            cls = rules.fallback;
        }
        status[obj] = st;
        chi0[obj] = c0;
        if (sw_out) sw_out[obj] = swt;
        const int32_t slot = atomicAdd(&counts[cls], 1);
        objs[(int64_t)cls * n_obj + slot] = (int32_t)obj;
    }
}

// Shared time sampling: CSR offsets o*n for the n_obj objects and the times
// relative to their minimum (non-finite times are left for the prep status).
__global__ __launch_bounds__(256) void shared_layout_kernel(const double *__restrict__ t,
                                                            int64_t n, int64_t n_obj,
                                                            int64_t *__restrict__ offsets,
                                                            double *__restrict__ shared_tt) {
    __shared__ double part[256 / kWave];
    const int tid = threadIdx.x;
    for (int64_t o = tid; o <= n_obj; o += 256) offsets[o] = o * n;
    double m = __builtin_inf();
    for (int64_t i = tid; i < n; i += 256) m = fmin(m, t[i]);
    m = wave_min(m);
    if (tid % kWave == 0) part[tid / kWave] = m;
    __syncthreads();
    double tmin = part[0];
    for (int w = 1; w < 256 / kWave; ++w) tmin = fmin(tmin, part[w]);
    for (int64_t i = tid; i < n; i += 256) shared_tt[i] = t[i] - tmin;
}

// One thread per object: first maximum over the tiles in frequency order,
// NaN skipped.
__global__ void finalize_kernel(const double *__restrict__ part_p,
                                const int32_t *__restrict__ part_k, int64_t n_obj,
                                int32_t n_tiles, const int32_t *__restrict__ status, double fmin,
                                double df, int64_t *__restrict__ best_idx,
                                double *__restrict__ best_period,
                                double *__restrict__ best_power) {
    const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= n_obj) return;
    double bp = 0.0;
    int64_t bk = -1;
    if (status[o] == 0) {
        for (int32_t i = 0; i < n_tiles; ++i) {
            int64_t q = o * n_tiles + i;
            int32_t k = part_k[q];
            double p = part_p[q];
            if (k < 0 || __builtin_isnan(p)) continue;
            if (bk < 0 || p > bp) {
                bp = p;
                bk = k;
            }
        }
    }
    if (best_idx) best_idx[o] = bk;
    if (bk >= 0) {
        double f = grid_freq(fmin, df, bk);
        if (best_period) best_period[o] = 1.0 / f;
        if (best_power) best_power[o] = bp;
    } else {
        if (best_period) best_period[o] = __builtin_nan("");
        if (best_power) best_power[o] = __builtin_nan("");
    }
}

}  // namespace

hipError_t launch_reset(int32_t *counts, unsigned long long *queues, int n, hipStream_t stream) {
    hipLaunchKernelGGL(reset_kernel, dim3(1), dim3(64), 0, stream, counts, queues, n);
    return hipGetLastError();
}

hipError_t launch_prep(const int64_t *offsets, const double *t, const double *y, const double *e,
                       int64_t n_obj, int64_t n_points, double *tt, double *w, double *yc, float *w32, float *yc32,
                       double *chi0, double *sw, int32_t *status, const ShapeRules &rules,
                       int32_t *objs, int32_t *counts, hipStream_t stream, bool shared_t) {
    if (n_obj <= 0) return hipSuccess;
    const int64_t blocks = (n_obj + kPrepWaves - 1) / kPrepWaves;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)blocks), dim3(kWave * kPrepWaves), 0, stream,
                       offsets, t, y, e, n_obj, n_points, tt, w, yc, w32, yc32, chi0, sw, status,
                       rules, objs, counts, shared_t ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_shared_layout(const double *t, int64_t n, int64_t n_obj, int64_t *offsets,
                                double *shared_tt, hipStream_t stream) {
    if (n_obj <= 0) return hipSuccess;
    hipLaunchKernelGGL(shared_layout_kernel, dim3(1), dim3(256), 0, stream, t, n, n_obj, offsets,
                       shared_tt);
    return hipGetLastError();
}

hipError_t launch_finalize(const double *part_p, const int32_t *part_k, int64_t n_obj,
                           int32_t n_tiles, const int32_t *status, double fmin, double df,
                           int64_t *best_idx, double *best_period, double *best_power,
                           hipStream_t stream) {
    if (n_obj <= 0) return hipSuccess;
    const int threads = 256;
    const int64_t blocks = (n_obj + threads - 1) / threads;
    hipLaunchKernelGGL(finalize_kernel, dim3((unsigned)blocks), dim3(threads), 0, stream, part_p,
                       part_k, n_obj, n_tiles, status, fmin, df, best_idx, best_period,
                       best_power);
    return hipGetLastError();
}

}  // namespace ssg
