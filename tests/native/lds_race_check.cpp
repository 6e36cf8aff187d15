// Runs the trial kernels' own source on the CPU, one OS thread per lane,
// against the CPU stand-in for HIP in tests/native/emu (built with
// ThreadSanitizer by tests/test_lds_race_cpu.py): every LDS read and write
// of a workgroup is then checked for an access of another lane that no
// barrier orders against it (a read that need not see its intended writer),
// while each group shape's wavefronts run in whatever order the OS gives
// them between barriers.  The periodograms are also compared with the CPU
// oracle.  Shapes include 2x4, which once gave wrong periodograms on the GPU
// in an earlier build.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <thread>
#include <vector>

#include "trial_impl.hpp"

extern "C" {
int ora_prep(int64_t n, const double *t, const double *y, const double *e, double *tt, double *w,
             double *ybar_out, double *chi0_out);
void ora_periodogram(int method, int64_t n_obj, const int64_t *offsets, const double *t,
                     const double *y, const double *e, double fmin, double fmax, int64_t n_freq,
                     const int64_t *ks, int64_t nk, const double *spans, double alpha,
                     double fixed_span, double *pgram, int32_t *status);
}

// the kernels' dynamic LDS array (declared in their namespace)
namespace ssg {
namespace {
alignas(16) unsigned char lds[192 * 1024];
}  // namespace
}  // namespace ssg
using ssg::lds;
namespace emu {
Group *g_group = nullptr;
thread_local int t_lane = 0, t_wave = 0;
}  // namespace emu
thread_local emu_dim3 threadIdx;
emu_dim3 blockIdx{0, 0, 0}, gridDim{1, 1, 1}, blockDim{64, 1, 1};

struct Catalog {
    std::vector<int64_t> offs{0};
    std::vector<double> t, y, e;
};

static uint64_t g_rng = 0x2545f4914f6cdd1dull;
static double uni() {
    g_rng = g_rng * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(g_rng >> 11) * 0x1p-53;
}

// kind 0 plain, 1 repeated times (exact ties), 2 a few points of tiny error
static void add_object(Catalog &c, int n, int kind) {
    double tc = 0.0;
    const double p = 0.3 + 4.0 * uni();
    for (int i = 0; i < n; ++i) {
        const double t = (kind == 1 && i % 3 == 2) ? c.t.back() : (tc += 0.2 + 5.0 * uni());
        c.t.push_back(t);
        c.y.push_back(15.0 + 0.3 * std::sin(6.283185307179586 * t / p) + 0.05 * (uni() - 0.5));
        c.e.push_back((kind == 2 && i % 17 == 3) ? 0.0003 : 0.02 + 0.05 * uni());
    }
    c.offs.push_back((int64_t)c.t.size());
}

static int g_fail = 0, g_cases = 0;

template <class P, int NW, int PPL, int M>
static void run_case(const Catalog &c, int64_t nf, int tile, const double spans[3], double alpha,
                     double fixed) {
    using namespace ssg;
    constexpr int NT = kWave * NW, NP = NT * PPL;
    const int64_t n_obj = (int64_t)c.offs.size() - 1, total = c.offs.back();
    std::vector<double> tt(total), w(total), yc(total), chi0(n_obj);
    std::vector<float> w32(total), yc32(total);
    std::vector<int32_t> status(n_obj), objs(n_obj);
    for (int64_t o = 0; o < n_obj; ++o) {
        const int64_t a = c.offs[o], n = c.offs[o + 1] - a;
        double ybar = 0.0;
        status[o] = ora_prep(n, &c.t[a], &c.y[a], &c.e[a], &tt[a], &w[a], &ybar, &chi0[o]);
        for (int64_t i = a; i < a + n; ++i) {
            yc[i] = c.y[i] - ybar;
            w32[i] = (float)w[i];
            yc32[i] = (float)yc[i];
        }
        objs[o] = (int32_t)o;
    }
    const int32_t count = (int32_t)n_obj;
    unsigned long long queues[kQueuesPerClass] = {};
    const double fmin = 0.1, fmax = 6.0;
    std::vector<double> pg(n_obj * nf, -7.0), po(n_obj * nf);
    TrialLaunch L{};
    L.cat = Prepared{c.offs.data(), tt.data(), w.data(), yc.data(), w32.data(), yc32.data(),
                     chi0.data(), status.data()};
    L.objs = objs.data();
    L.count = &count;
    L.queue = queues;
    L.tile_f = tile;
    L.n_tiles = (int32_t)((nf + tile - 1) / tile);
    L.fmin = fmin;
    L.df = (fmax - fmin) / (double)nf;
    L.n_freq = nf;
    for (int k = 0; k < 3; ++k) L.span[k] = spans[k];
    L.alpha = alpha;
    L.fixed_span = fixed;
    L.method = M;
    L.ext = std::max(2, halfwidth(NP, std::max(spans[2], fixed)));
    L.pgram64 = pg.data();
    if (Layout(NW, PPL, L.ext, M).bytes > (int)sizeof(lds)) {
        std::printf("skip %dx%d m%d: LDS\n", NW, PPL, M);
        return;
    }
    emu::Group G;
    G.nt = NT;
    G.bar.n = NT;
    G.waves = std::vector<emu::Wave>(NW);
    for (auto &wv : G.waves) {
        wv.bar.n = kWave;
        std::memset(wv.turn, 0, sizeof(wv.turn));
    }
    emu::g_group = &G;
    blockDim.x = NT;
    std::vector<std::thread> th;
    for (int t = 0; t < NT; ++t)
        th.emplace_back([&L, t] {
            threadIdx.x = (unsigned)t;
            emu::t_lane = t % kWave;
            emu::t_wave = t / kWave;
            trial_kernel<P, NW, PPL, M, false, false>(L);
        });
    for (auto &x : th) x.join();
    std::vector<int32_t> st(n_obj);
    ora_periodogram(M, n_obj, c.offs.data(), c.t.data(), c.y.data(), c.e.data(), fmin, fmax, nf,
                    nullptr, 0, spans, alpha, fixed, po.data(), st.data());
    // the FP64 parity bar, or the compensated-FP32 one (1e-2 everywhere)
    const double tol = P::kIsF64 ? 1e-4 : 1e-2;
    double worst = 0.0;
    int bad = 0;
    for (int64_t i = 0; i < n_obj * nf; ++i) {
        if (std::isnan(po[i]) != std::isnan(pg[i])) {
            ++bad;
            continue;
        }
        if (std::isnan(po[i])) continue;
        const double r = std::fabs(pg[i] - po[i]) / std::max(1.0 - po[i], 1e-12);
        worst = std::max(worst, r);
        bad += r > tol;
    }
    ++g_cases;
    if (bad) ++g_fail;
    std::printf("%s %dx%d method %d fixed %.2f: %lld trials, %d over %.0e, worst %.2e\n",
                P::kIsF64 ? "FP64" : "FP32c", NW, PPL, M, fixed, (long long)(n_obj * nf), bad, tol,
                worst);
    std::fflush(stdout);
}

template <int NW, int PPL>
static void run_shape() {
    constexpr int NP = 64 * NW * PPL;
    Catalog c;
    add_object(c, std::max(5, (int)(0.85 * NP)), 0);
    add_object(c, std::max(5, (int)(0.55 * NP)), 1);
    add_object(c, std::max(5, (int)(0.7 * NP)), 2);
    const double spans[3] = {0.05, 0.2, 0.5};
    // four frequencies, one per work item: more items than the one workgroup,
    // so it runs several in a row
    run_case<ssg::F64, NW, PPL, 0>(c, 4, 1, spans, 9.0, 0.0);
    run_case<ssg::F64, NW, PPL, 1>(c, 4, 1, spans, 9.0, 0.0);
    run_case<ssg::F64, NW, PPL, 2>(c, 4, 1, spans, 9.0, 0.0);
    run_case<ssg::F64, NW, PPL, 0>(c, 2, 1, spans, 9.0, 0.3);
    if constexpr (NW * PPL == 4) {  // the compensated-FP32 policy on the N=200 shapes
        run_case<ssg::F32C, NW, PPL, 0>(c, 3, 1, spans, 9.0, 0.0);
        run_case<ssg::F32C, NW, PPL, 1>(c, 3, 1, spans, 9.0, 0.0);
    }
}

// A planted mistake, to show that the harness reports one: two wavefronts,
// each lane writes its LDS word and then reads another wavefront's word with
// (ordered = 1) or without (ordered = 0) a workgroup barrier between.
static void planted(int ordered) {
    constexpr int NT = 128;
    emu::Group G;
    G.nt = NT;
    G.bar.n = NT;
    G.waves = std::vector<emu::Wave>(2);
    for (auto &wv : G.waves) {
        wv.bar.n = 64;
        std::memset(wv.turn, 0, sizeof(wv.turn));
    }
    emu::g_group = &G;
    std::vector<std::thread> th;
    unsigned sum = 0;
    std::mutex m;
    for (int t = 0; t < NT; ++t)
        th.emplace_back([&, t] {
            threadIdx.x = (unsigned)t;
            emu::t_lane = t % 64;
            emu::t_wave = t / 64;
            lds[t] = (unsigned char)t;
            if (ordered) __syncthreads();
            const unsigned v = lds[(t + 64) % NT];
            std::lock_guard<std::mutex> lk(m);
            sum += v;
        });
    for (auto &x : th) x.join();
    std::printf("planted (%s): sum %u\n", ordered ? "ordered" : "unordered", sum);
}

int main(int argc, char **argv) {
    if (argc > 1 && std::strcmp(argv[1], "plant") == 0) {
        planted(argc > 2 ? std::atoi(argv[2]) : 0);
        return 0;
    }
    const int big = argc > 1 ? std::atoi(argv[1]) : 0;
    run_shape<1, 1>();
    run_shape<1, 2>();
    run_shape<2, 1>();
    run_shape<1, 3>();
    run_shape<2, 2>();
    run_shape<1, 4>();
    run_shape<4, 1>();
    run_shape<2, 3>();
    run_shape<2, 4>();  // miscomputed in an earlier build
    run_shape<4, 2>();
    if (big) {
        run_shape<4, 4>();
        run_shape<8, 2>();
    }
    std::printf("emulated cases: %d, over tolerance: %d\n", g_cases, g_fail);
    return g_fail == 0 ? 0 : 1;
}
