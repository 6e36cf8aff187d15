// Per-object preparation (Alg. 1, compute_chi0_tt_weights) and the final
// per-object argmax over tile partials (Alg. 1, findPeriod).
#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

constexpr int kPrepWaves = 4;

// One wavefront per object.  FP64 throughout.  Status precedence: fewer than
// 5 points, non-finite t or y, bad error bar, chi0 == 0.
__global__ __launch_bounds__(kWave *kPrepWaves) void prep_kernel(
    const int64_t *__restrict__ offsets, const double *__restrict__ t,
    const double *__restrict__ y, const double *__restrict__ e, int64_t n_obj,
    double *__restrict__ tt, double *__restrict__ w, double *__restrict__ yc,
    float *__restrict__ w32, float *__restrict__ yc32, double *__restrict__ chi0,
    int32_t *__restrict__ status) {
    const int lane = threadIdx.x % kWave;
    const int64_t obj = (int64_t)blockIdx.x * kPrepWaves + threadIdx.x / kWave;
    if (obj >= n_obj) return;
    const int64_t a = offsets[obj], n = offsets[obj + 1] - a;
    if (n < 5) {
        if (lane == 0) {
            status[obj] = 1;
            chi0[obj] = __builtin_nan("");
        }
        return;
    }
    bool nonfinite = false, baderr = false;
    double tmin = __builtin_inf(), sw = 0.0, swy = 0.0;
    for (int64_t i = lane; i < n; i += kWave) {
        double ti = t[a + i], yi = y[a + i], ei = e[a + i];
        nonfinite |= !__builtin_isfinite(ti) || !__builtin_isfinite(yi);
        baderr |= !__builtin_isfinite(ei) || !(ei > 0.0);
        tmin = fmin(tmin, ti);
        double wi = 1.0 / (ei * ei);
        sw += wi;
        swy += wi * yi;
    }
    nonfinite = wave_ballot(nonfinite) != 0;
    baderr = wave_ballot(baderr) != 0;
    int32_t st = nonfinite ? 3 : (baderr ? 2 : 0);
    if (st != 0) {
        if (lane == 0) {
            status[obj] = st;
            chi0[obj] = __builtin_nan("");
        }
        return;
    }
    tmin = wave_min(tmin);
    sw = wave_sum(sw);
    swy = wave_sum(swy);
    const double ybar = swy / sw;
    double c0 = 0.0;
    for (int64_t i = lane; i < n; i += kWave) {
        double ei = e[a + i];
        double wi = 1.0 / (ei * ei);
        double d = y[a + i] - ybar;
        c0 += wi * d * d;
        tt[a + i] = t[a + i] - tmin;
        w[a + i] = wi;
        yc[a + i] = d;
        w32[a + i] = (float)wi;
        yc32[a + i] = (float)d;
    }
    c0 = wave_sum(c0);
    if (lane == 0) {
        status[obj] = (c0 > 0.0) ? 0 : 4;
        chi0[obj] = c0;
    }
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

hipError_t launch_prep(const int64_t *offsets, const double *t, const double *y, const double *e,
                       int64_t n_obj, double *tt, double *w, double *yc, float *w32, float *yc32,
                       double *chi0, int32_t *status, hipStream_t stream) {
    if (n_obj <= 0) return hipSuccess;
    const int64_t blocks = (n_obj + kPrepWaves - 1) / kPrepWaves;
    hipLaunchKernelGGL(prep_kernel, dim3((unsigned)blocks), dim3(kWave * kPrepWaves), 0, stream,
                       offsets, t, y, e, n_obj, tt, w, yc, w32, yc32, chi0, status);
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
