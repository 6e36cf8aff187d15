// Wavefront primitives for gfx950 (64 lanes): DPP prefix scans, lane reads,
// ballots and the wave-local LDS ordering barrier.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssg {

constexpr int kWave = 64;

// Orders this wave's LDS accesses across lanes: the LDS unit executes one
// wave's requests in issue order, so only compiler motion has to be stopped.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t wave_ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// DPP controls (gfx9 encoding): row_shr:n = 0x110+n, row_bcast:15 = 0x142,
// row_bcast:31 = 0x143.
template <int CTRL, int ROWMASK, bool BC>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWMASK, 0xf, BC);
}

template <int CTRL, int ROWMASK, bool BC>
__device__ __forceinline__ double dpp_f64(double v) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    int lo = dpp_i32<CTRL, ROWMASK, BC>((int)(uint32_t)u);
    int hi = dpp_i32<CTRL, ROWMASK, BC>((int)(uint32_t)(u >> 32));
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

template <int CTRL, int ROWMASK, bool BC>
__device__ __forceinline__ float dpp_f32(float v) {
    return __builtin_bit_cast(float, dpp_i32<CTRL, ROWMASK, BC>(__builtin_bit_cast(int, v)));
}

// Inclusive prefix sum over the 64 lanes (lane i gets the sum of lanes 0..i):
// four in-row shifts, then the row-15 and row-31 broadcasts.
__device__ __forceinline__ double wave_incl_sum(double x) {
    x += dpp_f64<0x111, 0xf, true>(x);
    x += dpp_f64<0x112, 0xf, true>(x);
    x += dpp_f64<0x114, 0xf, true>(x);
    x += dpp_f64<0x118, 0xf, true>(x);
    x += dpp_f64<0x142, 0xa, false>(x);
    x += dpp_f64<0x143, 0xc, false>(x);
    return x;
}

// The same scan with the two cross-row steps writing into caller-held
// temporaries z15, z31 that start at 0.0: a row_bcast step writes only the
// rows it adds to (rows 1, 3 and rows 2, 3), so the other rows of its
// temporary stay 0 from one scan to the next and need no clearing.  Every
// lane must be active (an inactive source lane would leave a stale value).
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dpp_f64_into(double old, double v) {
    const uint64_t uo = __builtin_bit_cast(uint64_t, old), uv = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)uo, (int)(uint32_t)uv, CTRL,
                                               ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(uo >> 32), (int)(uint32_t)(uv >> 32),
                                               CTRL, ROWMASK, 0xf, false);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ double wave_incl_sum_z(double x, double &z15, double &z31) {
    x += dpp_f64<0x111, 0xf, true>(x);
    x += dpp_f64<0x112, 0xf, true>(x);
    x += dpp_f64<0x114, 0xf, true>(x);
    x += dpp_f64<0x118, 0xf, true>(x);
    z15 = dpp_f64_into<0x142, 0xa>(z15, x);
    x += z15;
    z31 = dpp_f64_into<0x143, 0xc>(z31, x);
    x += z31;
    return x;
}

// M independent scans step by step (the in-row steps of all M first, so
// that their dependency chains overlap; the two cross-row steps pass the
// temporaries from one value to the next).
template <int M>
__device__ __forceinline__ void wave_incl_sum_z_multi(double (&x)[M], double &z15, double &z31) {
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] += dpp_f64<0x111, 0xf, true>(x[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] += dpp_f64<0x112, 0xf, true>(x[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] += dpp_f64<0x114, 0xf, true>(x[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) x[m] += dpp_f64<0x118, 0xf, true>(x[m]);
#pragma unroll
    for (int m = 0; m < M; ++m) {
        z15 = dpp_f64_into<0x142, 0xa>(z15, x[m]);
        x[m] += z15;
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
        z31 = dpp_f64_into<0x143, 0xc>(z31, x[m]);
        x[m] += z31;
    }
}

__device__ __forceinline__ uint32_t wave_incl_sum_u32(uint32_t v) {
    int x = (int)v;
    x += dpp_i32<0x111, 0xf, true>(x);
    x += dpp_i32<0x112, 0xf, true>(x);
    x += dpp_i32<0x114, 0xf, true>(x);
    x += dpp_i32<0x118, 0xf, true>(x);
    x += dpp_i32<0x142, 0xa, false>(x);
    x += dpp_i32<0x143, 0xc, false>(x);
    return (uint32_t)x;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
    uint64_t u = __builtin_bit_cast(uint64_t, v);
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, lane);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ float readlane_f32(float v, int lane) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), lane));
}

// Sum over the wave, identical in every lane.
__device__ __forceinline__ double wave_sum(double x) { return readlane_f64(wave_incl_sum(x), 63); }

__device__ __forceinline__ double wave_min(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmin(x, __shfl_xor(x, off, 64));
    return x;
}

__device__ __forceinline__ double wave_max(double x) {
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off, 64));
    return x;
}

}  // namespace ssg
