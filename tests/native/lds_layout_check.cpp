// Host-side bounds check of the trial kernels' LDS use, for every built
// shape, method, precision, span set (default and other spans, fixed spans)
// and every light-curve length a shape takes: the index ranges that the
// kernels' code reaches (listed per region below, with the function that
// reaches them) must lie inside the regions of the layout the kernels
// compute, and the regions must not overlap.  Built host-only against the
// kernels' own header (Layout, qaddr, halfwidth, prefix_arrays are the same
// code the device runs); run by tests/test_lds_layout_cpu.py.
#include <algorithm>
#include <cstdio>
#include <vector>

#include "trial_impl.hpp"

using namespace ssg;

static long n_fail = 0, n_checked = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        ++n_checked;                                      \
        if (!(cond)) {                                    \
            if (n_fail < 20) {                            \
                std::printf("FAIL %s: ", #cond);          \
                std::printf(__VA_ARGS__);                 \
                std::printf("\n");                        \
            }                                             \
            ++n_fail;                                     \
        }                                                 \
    } while (0)

template <int F, int PPL>
static int max_value_index(int slot_hi) {
    // qaddr grows with the slot; the last field of the highest slot
    return qaddr<F, PPL>(slot_hi) + F - 1;
}

template <int NW, int PPL>
static void check_shape(const double spans[3], double fixed) {
    const int np = kWave * NW * PPL;
    // the host's extension per class (api.hip, prepare): the half-width of
    // the largest span in use at the class's largest length
    const double span_hi = std::max(spans[2], fixed);
    const int ext = std::max(2, halfwidth(np, span_hi));
    for (int method = 0; method < 3; ++method) {
        const Layout Y(NW, PPL, ext, method);
        const int qvals = Y.qbytes / 8;  // S is 8 bytes in both policies
        // regions in order, no overlap (Layout)
        CHECK(Y.qbytes <= Y.sk && Y.sk % 16 == 0, "shape %dx%d m%d", NW, PPL, method);
        CHECK(Y.sk + np * 8 <= Y.xch, "SK region %dx%d", NW, PPL);
        CHECK(Y.xch + NW * 8 * 8 <= Y.qslot, "exchange region %dx%d", NW, PPL);
        CHECK(Y.qslot + 16 <= Y.best, "queue slot %dx%d", NW, PPL);
        CHECK(Y.best + kMaxSharedBatch * 12 <= Y.obj, "batch maxima %dx%d", NW, PPL);
        CHECK(Y.obj + (caches_object(np) ? 3 * np * 8 : 0) <= Y.cnt, "object cache %dx%d", NW, PPL);
        CHECK(Y.cnt + (np + 1) * 4 <= Y.bytes, "sort counters %dx%d", NW, PPL);
        // the sort's bucketed keys (fold_sort: tmp at the prefix region's
        // start, np keys, read by the ranking up to index np + kRankU - 1)
        // and the three scratch arrays of np values of the rare paths
        // (tie_average, cv_fallback: 8-byte FP64, 4-byte FP32)
        CHECK((np + kRankU) * 8 <= Y.qbytes, "bucketed keys %dx%d", NW, PPL);
        CHECK(3 * np * 8 <= Y.qbytes, "scratch %dx%d", NW, PPL);
        // exchange slots (8 NW doubles): group_excl of a build with offset
        // XO and M values up to 4 NW + 2 NW (the phase-A y build), the
        // chi^2 sum at 3 NW .. 4 NW, group_sum2 at 0 .. 2 NW
        CHECK(6 * NW <= 8 * NW, "exchange slots %dx%d", NW, PPL);
        for (int n = 5; n <= np; ++n) {
            const int b0 = halfwidth(n, spans[0]), b1 = halfwidth(n, spans[1]),
                      b2 = halfwidth(n, spans[2]);
            const int bf = fixed > 0.0 ? halfwidth(n, fixed) : 0;
            // half-widths and extensions the kernels use at this length:
            // supersmoother (b0, b1, b2; phase A extended by b2, phase B by
            // max(b0, b1); fixed: bf), single_pass (max over its spans)
            int bmax = fixed > 0.0 ? bf : std::max(b0, std::max(b1, b2));
            CHECK(bmax <= ext, "half-width %d > ext %d (%dx%d n=%d)", bmax, ext, NW, PPL, n);
            // slots reached: window ends at(j + b + 1) for j <= n - 1 (padding
            // lanes are clamped to n - 1) and at(j - b) for j >= 0, the
            // extension's copies at(n + u) (u <= e) and at(u - n) (u >= n - e);
            // at(i) is slot ext + i
            const int slot_lo = ext - bmax, slot_hi = ext + n + bmax;
            CHECK(slot_lo >= 0, "slot %d < 0 (%dx%d n=%d)", slot_lo, NW, PPL, n);
            const int F = Y.F;
            const int vi = F == 5 ? max_value_index<5, PPL>(slot_hi)
                                  : max_value_index<3, PPL>(slot_hi);
            CHECK(vi < qvals, "value %d >= %d (%dx%d m%d n=%d ext=%d)", vi, qvals, NW, PPL, method,
                  n, ext);
        }
    }
}

int main() {
    const double sets[4][3] = {{0.05, 0.2, 0.5}, {0.02, 0.1, 0.3}, {0.1, 0.3, 0.6},
                               {0.05, 0.2, 1.0}};
    const double fixeds[3] = {0.0, 0.3, 1.0};
    for (const auto &s : sets)
        for (double fx : fixeds) {
#define SSG_CHECK_SHAPE(nw, ppl) check_shape<nw, ppl>(s, fx);
            SSG_SHAPES(SSG_CHECK_SHAPE)
#undef SSG_CHECK_SHAPE
        }
    // which shapes fit the LDS of a CU (160 KB) at the default spans
    int fits = 0;
    for (int i = 0; i < kNumShapes; ++i) {
        const int np = kWave * kShapes[i].nw * kShapes[i].ppl;
        const int ext = std::max(2, halfwidth(np, 0.5));
        const Layout Y(kShapes[i].nw, kShapes[i].ppl, ext, 0);
        fits += Y.bytes <= 160 * 1024;
    }
    std::printf("lds layout: %ld checks, %ld failures, %d of %d shapes fit 160 KB at the default "
                "spans\n",
                n_checked, n_fail, fits, kNumShapes);
    return n_fail == 0 ? 0 : 1;
}
