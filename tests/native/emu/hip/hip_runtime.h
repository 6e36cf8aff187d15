// A CPU stand-in for the parts of the HIP runtime and of the gfx950
// builtins that the trial kernels use, so that the kernels' own source can
// be compiled for the host and run by one OS thread per lane (test
// infrastructure: tests/native/lds_race_check.cpp).  Barriers are mutex and
// condition-variable rendezvous, so ThreadSanitizer sees exactly the
// ordering that the kernels' barriers give; cross-lane builtins (DPP moves,
// lane reads, ballots) exchange values through per-wavefront slots between
// two wavefront rendezvous.  LDS is one process-wide array (one workgroup
// runs at a time).
#pragma once
#include <atomic>
#include <condition_variable>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <vector>

#define __host__
#define __device__
#define __global__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__
#define __align__(x) alignas(x)

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2 };
typedef void *hipStream_t;
enum hipFuncAttribute { hipFuncAttributeMaxDynamicSharedMemorySize = 8 };
inline hipError_t hipFuncSetAttribute(const void *, hipFuncAttribute, int) { return hipSuccess; }
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *n, const void *, int, size_t) {
    *n = 1;
    return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "emulated"; }
struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};
// launches are made by the emulator's driver, not through this macro
#define hipLaunchKernelGGL(kernel, grid, block, lds_bytes, stream, ...) ((void)0)

namespace emu {

struct Rendezvous {
    // counting barrier on one atomic word (C++20 wait/notify); the
    // acquire/release pairs give ThreadSanitizer the barrier's ordering
    std::atomic<unsigned> arrived{0}, gen{0};
    int n = 0;
    void wait() {
        const unsigned g = gen.load(std::memory_order_acquire);
        if (arrived.fetch_add(1, std::memory_order_acq_rel) + 1 == (unsigned)n) {
            arrived.store(0, std::memory_order_relaxed);
            gen.fetch_add(1, std::memory_order_acq_rel);
            gen.notify_all();
        } else {
            unsigned cur;
            while ((cur = gen.load(std::memory_order_acquire)) == g) gen.wait(g);
        }
    }
};

struct Wave {
    Rendezvous bar;
    int64_t slot[2][64];  // exchange buffers used in turn
    unsigned turn[64];    // per lane: which buffer its next exchange uses
};

struct Group {
    int nt = 0;
    Rendezvous bar;
    std::vector<Wave> waves;
    std::mutex or_m;
    int or_acc[2] = {0, 0};
    unsigned or_phase = 0;
};

extern Group *g_group;
extern thread_local int t_lane, t_wave;
unsigned threadIdx_x();

inline Wave &wave() { return g_group->waves[(size_t)t_wave]; }

// value of another lane of this wavefront (all lanes take part).  One
// rendezvous per exchange: consecutive exchanges use the two buffers in
// turn, and a buffer is written again only after every lane has passed the
// next exchange's rendezvous, i.e. finished reading it.
inline int64_t exchange(int64_t v, int src_lane, bool &valid) {
    Wave &w = wave();
    const unsigned b = w.turn[t_lane] & 1u;
    w.turn[t_lane]++;
    w.slot[b][t_lane] = v;
    w.bar.wait();
    valid = src_lane >= 0 && src_lane < 64;
    return valid ? w.slot[b][src_lane] : 0;
}

// DPP move of gfx9: row_shr:n (0x111..0x11f), row_bcast:15 (0x142),
// row_bcast:31 (0x143); rows outside row_mask keep `old`; an invalid source
// gives 0 with bound_ctrl, else `old`
inline int update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    if (bank_mask != 0xf) std::abort();
    const int l = t_lane, row = l / 16, lr = l % 16;
    int s = -1;
    if (ctrl >= 0x111 && ctrl <= 0x11f) {
        const int k = ctrl - 0x110;
        s = lr >= k ? l - k : -1;
    } else if (ctrl == 0x142) {
        s = row >= 1 ? row * 16 - 1 : -1;
    } else if (ctrl == 0x143) {
        s = row >= 2 ? 31 : -1;
    } else {
        std::abort();
    }
    bool valid = false;
    const int v = (int)exchange((int64_t)src, s, valid);
    if (!((row_mask >> row) & 1)) return old;
    if (!valid) return bound_ctrl ? 0 : old;
    return v;
}

inline int readlane(int v, int lane) {
    bool valid = false;
    return (int)exchange((int64_t)v, lane, valid);
}
inline int readfirstlane(int v) { return readlane(v, 0); }

inline uint64_t ballot(bool p) {
    Wave &w = wave();
    const unsigned b = w.turn[t_lane] & 1u;
    w.turn[t_lane]++;
    w.slot[b][t_lane] = p ? 1 : 0;
    w.bar.wait();
    uint64_t m = 0;
    for (int i = 0; i < 64; ++i)
        if (w.slot[b][i]) m |= 1ull << i;
    return m;
}

inline void wave_barrier() { wave().bar.wait(); }

inline void syncthreads() { g_group->bar.wait(); }

inline int syncthreads_or(int p) {
    Group &g = *g_group;
    unsigned ph;
    {
        std::lock_guard<std::mutex> lk(g.or_m);
        ph = g.or_phase & 1u;
        g.or_acc[ph] |= p ? 1 : 0;
    }
    g.bar.wait();
    int r;
    {
        std::lock_guard<std::mutex> lk(g.or_m);
        r = g.or_acc[ph];
    }
    g.bar.wait();
    // one thread resets the slot for the use after next
    if (threadIdx_x() == 0) {
        std::lock_guard<std::mutex> lk(g.or_m);
        g.or_acc[ph] = 0;
        g.or_phase++;
    }
    g.bar.wait();
    return r;
}

}  // namespace emu

struct emu_dim3 {
    unsigned x, y, z;
};
extern thread_local emu_dim3 threadIdx;
extern emu_dim3 blockIdx, gridDim, blockDim;
inline unsigned emu::threadIdx_x() { return threadIdx.x; }

#define __builtin_amdgcn_update_dpp(old, src, ctrl, rm, bm, bc) \
    emu::update_dpp((old), (src), (ctrl), (rm), (bm), (bc))
#define __builtin_amdgcn_readlane(v, l) emu::readlane((v), (l))
#define __builtin_amdgcn_readfirstlane(v) emu::readfirstlane((int)(v))
#define __builtin_amdgcn_ballot_w64(p) emu::ballot((p))
#define __builtin_amdgcn_wave_barrier() emu::wave_barrier()
#define __builtin_amdgcn_fence(order, scope) ((void)0)
#define __builtin_amdgcn_rcp(a) (1.0 / (a))
#define __builtin_amdgcn_rcpf(a) (1.0f / (a))
#define __builtin_amdgcn_exp2f(a) std::exp2((float)(a))
#define __builtin_amdgcn_logf(a) std::log2((float)(a))
#define __syncthreads() emu::syncthreads()
#define __syncthreads_or(p) emu::syncthreads_or((p))

// HIP's device min/max on integers and the wavefront shuffle
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline double __shfl_xor(double v, int mask, int width) {
    (void)width;
    bool valid = false;
    int64_t bits;
    std::memcpy(&bits, &v, 8);
    const int64_t r = emu::exchange(bits, emu::t_lane ^ mask, valid);
    double out;
    std::memcpy(&out, &r, 8);
    return out;
}

template <class T>
inline T atomicAdd(T *p, T v) {
    return __atomic_fetch_add(p, v, __ATOMIC_RELAXED);
}
