// Cheap exact-grid proposal for search-and-refine (Sec. 6 proposes
// refining around the peaks of a cheaper search).  For each (object, grid
// frequency) the light curve is folded in FP64 and its points are binned
// into B equal phase bins; the score is the fraction of chi0 explained by
// the bins' weighted means, sum_b (sum w yc)_b^2 / (sum w)_b / chi0 (yc is y
// minus the weighted mean, so the total mean term vanishes).  This is a
// phase-dispersion statistic: no sort, two LDS accumulations per point.
// Each lane owns one frequency and private bins laid out [bin][lane] (no
// bank conflicts, no atomics); the points are uniform across the wavefront.
// Scores are max-pooled into the grid's 1024 log bins with a wavefront
// segmented maximum and one global atomic maximum per segment.
#include <algorithm>

#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

constexpr int kWavesPerBlock = 4;

__global__ void zero_kernel(float *__restrict__ p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

__device__ __forceinline__ int log_bin_of(const int64_t *__restrict__ bin_k, int64_t k) {
    // largest b with bin_k[b] <= k (bin_k is non-decreasing, bin_k[0] = 0)
    int lo = 0, hi = kEncBins;  // invariant: bin_k[lo] <= k < bin_k[hi] (bin_k[1024] = n_freq)
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (bin_k[mid] <= k)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

__global__ __launch_bounds__(kWave *kWavesPerBlock) void bin_score_kernel(ScoreArgs A) {
    __shared__ float acc[kWavesPerBlock][2 * kScoreMaxBins][kWave];
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    float(*W)[kWave] = acc[wv];
    float(*S)[kWave] = acc[wv] + kScoreMaxBins;
    const int64_t chunks = (A.n_freq + kWave - 1) / kWave;
    const int64_t total = (int64_t)A.n_obj * chunks;
    const int64_t n_waves = (int64_t)gridDim.x * kWavesPerBlock;
    for (int64_t item = (int64_t)blockIdx.x * kWavesPerBlock + wv; item < total;
         item += n_waves) {
        const int o = (int)(item / chunks);
        const int64_t k = (item - (int64_t)o * chunks) * kWave + lane;
        if (A.status[o] != 0) continue;
        const int64_t a = A.offsets[o];
        const int n = (int)(A.offsets[o + 1] - a);
        const int B = min(kScoreMaxBins, max(4, n / 5));
        for (int b = 0; b < B; ++b) {
            W[b][lane] = 0.0f;
            S[b][lane] = 0.0f;
        }
        const bool live = k < A.n_freq;
        const double f = grid_freq(A.fmin, A.df, live ? k : 0);
        const double *tt = A.tt + a;
        const double *w = A.w + a;
        const double *yc = A.yc + a;
        for (int i = 0; i < n; ++i) {
            const double q = tt[i] * f;
            const double ph = q - floor(q);
            const int jb = min(B - 1, (int)(ph * (double)B));
            const float wi = (float)w[i];
            W[jb][lane] += wi;
            S[jb][lane] += wi * (float)yc[i];
        }
        float e = 0.0f;
        for (int b = 0; b < B; ++b) {
            const float wb = W[b][lane];
            if (wb > 0.0f) e += S[b][lane] * S[b][lane] / wb;
        }
        float score = live ? (float)((double)e / A.chi0[o]) : -1.0f;
        int lb = live ? log_bin_of(A.bin_k, k) : 0x7fffffff;
        // segmented maximum over lanes with the same log bin (non-decreasing in lane)
        for (int off = 1; off < kWave; off <<= 1) {
            const float os = __shfl_down(score, off);
            const int ob = __shfl_down(lb, off);
            if (lane + off < kWave && ob == lb) score = fmaxf(score, os);
        }
        const int prev = __shfl_up(lb, 1);
        if (live && (lane == 0 || prev != lb))
            atomicMax((int *)&A.scores[(int64_t)o * kEncBins + lb], __float_as_int(score));
    }
}

}  // namespace

hipError_t launch_bin_scores(const ScoreArgs &A, int n_cu, hipStream_t s) {
    if (A.n_obj <= 0) return hipSuccess;
    const int64_t n = (int64_t)A.n_obj * kEncBins;
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, A.scores,
                       n);
    const int64_t items = (int64_t)A.n_obj * ((A.n_freq + kWave - 1) / kWave);
    int64_t blocks = std::min<int64_t>((int64_t)n_cu * 8, (items + kWavesPerBlock - 1) /
                                                              kWavesPerBlock);
    hipLaunchKernelGGL(bin_score_kernel, dim3((unsigned)std::max<int64_t>(blocks, 1)),
                       dim3(kWave * kWavesPerBlock), 0, s, A);
    return hipGetLastError();
}

}  // namespace ssg
