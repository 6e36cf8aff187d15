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

// One launch of the trial kernel over one size class.
struct TrialLaunch {
    Prepared cat;
    const int32_t *objs;  // object ids of this class
    int64_t n_items;      // objects_in_class * n_tiles
    int32_t n_tiles;
    int32_t tile_f;
    double fmin, df;
    int64_t n_freq;
    double span[3];
    double alpha;
    double fixed_span;
    int32_t method;       // 0 SS, 1 SSSP
    double *pgram64;      // [n_obj * n_freq] or null
    float *pgram32;       // [n_obj * n_freq] or null
    double *part_p;       // [n_obj * n_tiles] or null
    int32_t *part_k;      // [n_obj * n_tiles] or null
};

// Expressions that must round exactly like their plain C statement (no
// fused multiply-add), so that grid frequencies, window half-widths and the
// Listing 1 threshold agree bit for bit with a straightforward evaluation.
__device__ __forceinline__ double grid_freq(double fmin, double df, int64_t k) {
#pragma clang fp contract(off)
    double kd = (double)k;
    double step = kd * df;
    return fmin + step;
}

__device__ __forceinline__ double halfwidth_real(double span, int n) {
#pragma clang fp contract(off)
    return 0.5 * span * (double)n + 0.5;
}

__device__ __forceinline__ double listing_vsmlsq(double scale) {
#pragma clang fp contract(off)
    return 1.0e-6 * scale * scale;
}

// Size classes: one wavefront per trial, PPL points per lane.
constexpr int kClassPPL[] = {1, 2, 3, 4, 6, 8};
constexpr int kNumClasses = 6;
constexpr int kMaxSingleWave = 64 * 8;

int class_of_length(int64_t n);  // index into kClassPPL, -1 if too long

hipError_t launch_prep(const int64_t *offsets, const double *t, const double *y, const double *e,
                       int64_t n_obj, double *tt, double *w, double *yc, float *w32, float *yc32,
                       double *chi0, int32_t *status, hipStream_t stream);

hipError_t launch_trials(int cls, int precision, const TrialLaunch &L, hipStream_t stream);

hipError_t launch_finalize(const double *part_p, const int32_t *part_k, int64_t n_obj,
                           int32_t n_tiles, const int32_t *status, double fmin, double df,
                           int64_t *best_idx, double *best_period, double *best_power,
                           hipStream_t stream);

}  // namespace ssg
