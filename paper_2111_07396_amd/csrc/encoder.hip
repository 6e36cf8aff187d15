// Learned frequency proposal: the set encoder that ranks log-spaced frequency
// bins for each light curve, its training kernels, and the refine planner
// that turns the top bins into fine-grid frequency ranges for the exact
// trial kernel.  This is the paper's proposed search-and-refine (Sec. 6),
// with a learned proposal in place of a cheap periodogram.
//
// Network, per object of n points (features of point i in 80 slots):
//   slots 2m, 2m+1 : sin, cos of 2 pi g_m tt_i, g_m log-spaced over the band
//   slots 64, 65   : (y_i - ybar)/sigma, e_i/sigma   (weighted mean / spread)
//   slot 66        : 1 (the first layer's bias is row 66 of W1)
//   a1 = x W1 [64], h1 = relu(a1), a2 = h1 W2 + b2 [128], h2 = relu(a2),
//   emb = mean_i h2, logits = emb W3 + b3 [1024].
// The two per-point layers run on the gfx950 BF16 matrix cores (32x32x16
// MFMA, FP32 accumulate) in the transposed form H^T = W^T X^T, so that the
// output of one layer is the B operand of the next without leaving
// registers (the contraction index may be permuted freely, so the weights
// are stored in LDS in the order the accumulator layout produces).  The
// weight gradients contract over points and go through a per-wave LDS
// transpose into 16x16x32 MFMAs.  The 1024-bin head is a small FP32 VALU
// GEMM.
#include <algorithm>

#include "ssgpu_internal.hpp"
#include "wave.hpp"

namespace ssg {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int K1 = kEncK1, H1 = kEncH1, H2 = kEncH2, NB = kEncBins;
constexpr int OFF_W1 = 0, OFF_W2 = K1 * H1, OFF_B2 = OFF_W2 + H1 * H2, OFF_W3 = OFF_B2 + H2,
              OFF_B3 = OFF_W3 + H2 * NB;
static_assert(OFF_B3 + NB == kEncParams, "parameter layout");
constexpr int kMlpGrad = K1 * H1 + H1 * H2;  // W1 and W2 gradient floats per wave partial

// LDS fragment tables (bf16x8 per lane): W1^T for layer 1 [mt 2][ks 5][64],
// W2^T for layer 2 [mt2 4][ks 4][64], W2 for the backward product [mt 2][ks 8][64].
constexpr int kW1f = 2 * 5 * 64, kW2f = 4 * 4 * 64, kW2b = 2 * 8 * 64;
constexpr int kPT = 40;  // row stride (bf16) of the per-wave transposed tiles
constexpr int kRowsT = K1 + H1 + H2 + H1;

__device__ __forceinline__ int c_row(int i, int g) {  // row of accumulator i (32x32 layout)
    return 8 * (i >> 2) + 4 * g + (i & 3);
}

__device__ __forceinline__ floatx16 mfma32(bf16x8 a, bf16x8 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ floatx4 mfma16(bf16x8 a, bf16x8 b, floatx4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Fills the weight fragment tables from the FP32 master parameters.
template <bool BWD>
__device__ void load_weights(const float *__restrict__ prm, bf16x8 *w1f, bf16x8 *w2f, float *b2s,
                             bf16x8 *w2b) {
    for (int idx = threadIdx.x; idx < kW1f; idx += blockDim.x) {
        const int mt = idx / 320, ks = (idx / 64) % 5, l = idx % 64, g = l / 32;
        const int h = 32 * mt + l % 32;
        bf16x8 v;
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)prm[OFF_W1 + (16 * ks + 8 * g + i) * H1 + h];
        w1f[idx] = v;
    }
    for (int idx = threadIdx.x; idx < kW2f; idx += blockDim.x) {
        const int mt2 = idx / 256, ks2 = (idx / 64) % 4, l = idx % 64, g = l / 32;
        const int u = 32 * mt2 + l % 32, mt = ks2 >> 1, half = ks2 & 1;
        bf16x8 v;
        for (int i = 0; i < 8; ++i) {
            const int h = 32 * mt + 16 * half + 8 * (i >> 2) + 4 * g + (i & 3);
            v[i] = (__bf16)prm[OFF_W2 + h * H2 + u];
        }
        w2f[idx] = v;
    }
    for (int idx = threadIdx.x; idx < H2; idx += blockDim.x) b2s[idx] = prm[OFF_B2 + idx];
    if (BWD) {
        for (int idx = threadIdx.x; idx < kW2b; idx += blockDim.x) {
            const int mt = idx / 512, ks = (idx / 64) % 8, l = idx % 64, g = l / 32;
            const int h = 32 * mt + l % 32, mt2 = ks >> 1, half = ks & 1;
            bf16x8 v;
            for (int i = 0; i < 8; ++i) {
                const int u = 32 * mt2 + 16 * half + 8 * (i >> 2) + 4 * g + (i & 3);
                v[i] = (__bf16)prm[OFF_W2 + h * H2 + u];
            }
            w2b[idx] = v;
        }
    }
}

struct PointCtx {
    const double *tt, *yc, *e;
    int n;
    float inv_sigma;
};

// B-operand fragment of the features for k-step ks (feature slots
// 16 ks + 8 g + 0..7) of point p; zero for padding points.
__device__ __forceinline__ bf16x8 feature_frag(const EncArgs &A, const PointCtx &P, int p, int ks,
                                               int g) {
    bf16x8 v;
    if (p >= P.n) {
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.0f;
        return v;
    }
    if (ks < 4) {
        const double tt = P.tt[p];
        for (int j = 0; j < 4; ++j) {
            const double q = tt * A.g[8 * ks + 4 * g + j];
            const float ph = (float)(q - floor(q));
            // the hardware sine/cosine take their argument in revolutions
            v[2 * j] = (__bf16)__builtin_amdgcn_sinf(ph);
            v[2 * j + 1] = (__bf16)__builtin_amdgcn_cosf(ph);
        }
    } else {
        for (int i = 0; i < 8; ++i) v[i] = (__bf16)0.0f;
        if (g == 0) {
            v[0] = (__bf16)((float)P.yc[p] * P.inv_sigma);
            v[1] = (__bf16)((float)P.e[p] * P.inv_sigma);
            v[2] = (__bf16)1.0f;
        }
    }
    return v;
}

// Sum over the 32 lanes that share g = lane / 32 of a 64-entry per-lane
// vector, as a butterfly reduce-scatter (62 shuffles): afterwards lane l
// holds entries 2 (l % 32) and 2 (l % 32) + 1.
__device__ __forceinline__ void reduce_scatter32(float (&v)[64], int lane) {
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        const int mask = 16 >> s, W = 64 >> s, Hh = W / 2;
        const bool hi = (lane & mask) != 0;
#pragma unroll
        for (int j = 0; j < Hh; ++j) {
            const float send = hi ? v[j] : v[j + Hh];
            const float keep = hi ? v[j + Hh] : v[j];
            v[j] = keep + __shfl_xor(send, mask);
        }
    }
}

__device__ __forceinline__ int reduced_unit(int j, int g) {  // u of entry j = 16 mt2 + i
    return 32 * (j >> 4) + c_row(j & 15, g);
}

__device__ __forceinline__ bool obj_setup(const EncArgs &A, int o, PointCtx &P) {
    if (A.status[o] != 0) return false;
    const int64_t a = A.offsets[o];
    P.n = (int)(A.offsets[o + 1] - a);
    P.tt = A.tt + a;
    P.yc = A.yc + a;
    P.e = A.e + a;
    P.inv_sigma = (float)(1.0 / sqrt(A.chi0[o] / A.sw[o]));
    return true;
}

// Forward: emb[o] = mean of h2, act[o] = fraction of points with a2 > 0 (when
// act is given).  One wavefront per object, persistent over objects.  Held to
// two wavefronts per SIMD, which it fits without spills (unbounded, the
// compiler keeps more in flight and allows only one).
__global__ __launch_bounds__(256, 2) void enc_fwd_kernel(EncArgs A) {
    extern __shared__ __align__(16) unsigned char lds[];
    bf16x8 *w1f = (bf16x8 *)lds;
    bf16x8 *w2f = w1f + kW1f;
    float *b2s = (float *)(w2f + kW2f);
    load_weights<false>(A.params, w1f, w2f, b2s, nullptr);
    __syncthreads();
    const int lane = threadIdx.x % kWave, g = lane / 32;
    const int waves = gridDim.x * (blockDim.x / kWave);
    for (int o = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; o < A.n_obj;
         o += waves) {
        PointCtx P;
        float acc[64], cnt[64];
        for (int j = 0; j < 64; ++j) acc[j] = cnt[j] = 0.0f;
        const bool ok = obj_setup(A, o, P);
        const int n = ok ? P.n : 0;
        for (int p0 = 0; p0 < n; p0 += 32) {
            const int p = p0 + lane % 32;
            floatx16 c1[2] = {};
#pragma unroll
            for (int ks = 0; ks < 5; ++ks) {
                const bf16x8 xf = feature_frag(A, P, p, ks, g);
                c1[0] = mfma32(w1f[(0 * 5 + ks) * 64 + lane], xf, c1[0]);
                c1[1] = mfma32(w1f[(1 * 5 + ks) * 64 + lane], xf, c1[1]);
            }
            bf16x8 hf[4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                    for (int i = 0; i < 8; ++i)
                        hf[2 * mt + hh][i] = (__bf16)fmaxf(c1[mt][8 * hh + i], 0.0f);
            const bool valid = p < n;
#pragma unroll
            for (int mt2 = 0; mt2 < 4; ++mt2) {
                floatx16 c2;
#pragma unroll
                for (int i = 0; i < 16; ++i) c2[i] = b2s[32 * mt2 + c_row(i, g)];
#pragma unroll
                for (int ks2 = 0; ks2 < 4; ++ks2)
                    c2 = mfma32(w2f[(mt2 * 4 + ks2) * 64 + lane], hf[ks2], c2);
                if (valid) {
#pragma unroll
                    for (int i = 0; i < 16; ++i) {
                        acc[16 * mt2 + i] += fmaxf(c2[i], 0.0f);
                        cnt[16 * mt2 + i] += c2[i] > 0.0f ? 1.0f : 0.0f;
                    }
                }
            }
        }
        reduce_scatter32(acc, lane);
        reduce_scatter32(cnt, lane);
        const float inv_n = n > 0 ? 1.0f / (float)n : 0.0f;
        for (int r = 0; r < 2; ++r) {
            const int u = reduced_unit(2 * (lane % 32) + r, g);
            A.emb[(int64_t)o * H2 + u] = acc[r] * inv_n;
            if (A.act) A.act[(int64_t)o * H2 + u] = cnt[r] * inv_n;
        }
    }
}

// Backward through the per-point layers for the loss gradient dE = dL/d emb
// (one wavefront per object, forward recomputed tile by tile).  Each wave
// accumulates its objects' W1 and W2 gradients in MFMA accumulators and
// writes them to its own partial slot; a reduction kernel sums the slots.
__global__ __launch_bounds__(128) void enc_bwd_kernel(EncArgs A) {
    extern __shared__ __align__(16) unsigned char lds[];
    bf16x8 *w1f = (bf16x8 *)lds;
    bf16x8 *w2f = w1f + kW1f;
    float *b2s = (float *)(w2f + kW2f);
    bf16x8 *w2b = (bf16x8 *)(b2s + H2);
    load_weights<true>(A.params, w1f, w2f, b2s, w2b);
    const int lane = threadIdx.x % kWave, g = lane / 32, wv = threadIdx.x / kWave;
    float *dEs = (float *)(w2b + kW2b) + wv * H2;
    __bf16 *tiles = (__bf16 *)((float *)(w2b + kW2b) + (blockDim.x / kWave) * H2) +
                    (size_t)wv * kRowsT * kPT;
    __bf16 *XT = tiles, *H1T = XT + K1 * kPT, *D2T = H1T + H1 * kPT, *D1T = D2T + H2 * kPT;
    __syncthreads();
    floatx4 gw2[4][8], gw1[5][4];
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 8; ++b) gw2[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    for (int a = 0; a < 5; ++a)
        for (int b = 0; b < 4; ++b) gw1[a][b] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int wave_id = blockIdx.x * (blockDim.x / kWave) + wv;
    const int waves = gridDim.x * (blockDim.x / kWave);
    for (int o = wave_id; o < A.n_obj; o += waves) {
        PointCtx P;
        if (!obj_setup(A, o, P)) continue;
        const int n = P.n;
        const float inv_n = 1.0f / (float)n;
        for (int u = lane; u < H2; u += kWave) dEs[u] = A.dE[(int64_t)o * H2 + u] * inv_n;
        wave_lds_sync();
        for (int p0 = 0; p0 < n; p0 += 32) {
            const int pc = lane % 32, p = p0 + pc;
            const bool valid = p < n;
            floatx16 c1[2] = {};
#pragma unroll
            for (int ks = 0; ks < 5; ++ks) {
                const bf16x8 xf = feature_frag(A, P, p, ks, g);
#pragma unroll
                for (int i = 0; i < 8; ++i) XT[(16 * ks + 8 * g + i) * kPT + pc] = xf[i];
                c1[0] = mfma32(w1f[(0 * 5 + ks) * 64 + lane], xf, c1[0]);
                c1[1] = mfma32(w1f[(1 * 5 + ks) * 64 + lane], xf, c1[1]);
            }
            bf16x8 hf[4];
#pragma unroll
            for (int mt = 0; mt < 2; ++mt)
#pragma unroll
                for (int hh = 0; hh < 2; ++hh)
#pragma unroll
                    for (int i = 0; i < 8; ++i) {
                        const __bf16 hv = (__bf16)fmaxf(c1[mt][8 * hh + i], 0.0f);
                        hf[2 * mt + hh][i] = hv;
                        H1T[(32 * mt + c_row(8 * hh + i, g)) * kPT + pc] = hv;
                    }
            bf16x8 df[8];
#pragma unroll
            for (int mt2 = 0; mt2 < 4; ++mt2) {
                floatx16 c2;
#pragma unroll
                for (int i = 0; i < 16; ++i) c2[i] = b2s[32 * mt2 + c_row(i, g)];
#pragma unroll
                for (int ks2 = 0; ks2 < 4; ++ks2)
                    c2 = mfma32(w2f[(mt2 * 4 + ks2) * 64 + lane], hf[ks2], c2);
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int u = 32 * mt2 + c_row(i, g);
                    const __bf16 dv = (__bf16)((valid && c2[i] > 0.0f) ? dEs[u] : 0.0f);
                    df[2 * mt2 + (i >> 3)][i & 7] = dv;
                    D2T[u * kPT + pc] = dv;
                }
            }
#pragma unroll
            for (int mt = 0; mt < 2; ++mt) {
                floatx16 d = {};
#pragma unroll
                for (int ks = 0; ks < 8; ++ks) d = mfma32(w2b[(mt * 8 + ks) * 64 + lane], df[ks], d);
#pragma unroll
                for (int i = 0; i < 16; ++i)
                    D1T[(32 * mt + c_row(i, g)) * kPT + pc] =
                        (__bf16)(c1[mt][i] > 0.0f ? d[i] : 0.0f);
            }
            wave_lds_sync();
            const int r = lane % 16, kq = 8 * (lane / 16);
            bf16x8 bh[4];
#pragma unroll
            for (int mh = 0; mh < 4; ++mh) bh[mh] = *(const bf16x8 *)&H1T[(16 * mh + r) * kPT + kq];
#pragma unroll
            for (int nu = 0; nu < 8; ++nu) {
                const bf16x8 bd = *(const bf16x8 *)&D2T[(16 * nu + r) * kPT + kq];
#pragma unroll
                for (int mh = 0; mh < 4; ++mh) gw2[mh][nu] = mfma16(bh[mh], bd, gw2[mh][nu]);
            }
            bf16x8 b1[4];
#pragma unroll
            for (int nh = 0; nh < 4; ++nh) b1[nh] = *(const bf16x8 *)&D1T[(16 * nh + r) * kPT + kq];
#pragma unroll
            for (int mk = 0; mk < 5; ++mk) {
                const bf16x8 bx = *(const bf16x8 *)&XT[(16 * mk + r) * kPT + kq];
#pragma unroll
                for (int nh = 0; nh < 4; ++nh) gw1[mk][nh] = mfma16(bx, b1[nh], gw1[mk][nh]);
            }
            wave_lds_sync();
        }
    }
    float *out = A.partial + (int64_t)wave_id * kMlpGrad;
    const int col = lane % 16, rq = 4 * (lane / 16);
    for (int mk = 0; mk < 5; ++mk)
        for (int nh = 0; nh < 4; ++nh)
            for (int i = 0; i < 4; ++i)
                out[(16 * mk + rq + i) * H1 + 16 * nh + col] = gw1[mk][nh][i];
    for (int mh = 0; mh < 4; ++mh)
        for (int nu = 0; nu < 8; ++nu)
            for (int i = 0; i < 4; ++i)
                out[K1 * H1 + (16 * mh + rq + i) * H2 + 16 * nu + col] = gw2[mh][nu][i];
}

// logits[o][b] = b3[b] + sum_k emb[o][k] W3[k][b]: 32 objects x 1024 bins per
// workgroup, 4 bins x 32 objects per thread.
constexpr int kHeadObj = 32;
__global__ __launch_bounds__(256) void head_fwd_kernel(const float *__restrict__ emb,
                                                       const float *__restrict__ prm, int n_obj,
                                                       float *__restrict__ logits) {
    __shared__ float es[kHeadObj][H2];
    const int o0 = blockIdx.x * kHeadObj;
    for (int i = threadIdx.x; i < kHeadObj * H2; i += blockDim.x) {
        const int o = o0 + i / H2;
        es[i / H2][i % H2] = o < n_obj ? emb[(int64_t)o * H2 + i % H2] : 0.0f;
    }
    __syncthreads();
    const int b = 4 * threadIdx.x;
    float acc[kHeadObj][4];
    const float4 bias = *(const float4 *)&prm[OFF_B3 + b];
    for (int o = 0; o < kHeadObj; ++o) {
        acc[o][0] = bias.x;
        acc[o][1] = bias.y;
        acc[o][2] = bias.z;
        acc[o][3] = bias.w;
    }
    for (int k = 0; k < H2; ++k) {
        const float4 wv = *(const float4 *)&prm[OFF_W3 + k * NB + b];
#pragma unroll
        for (int o = 0; o < kHeadObj; ++o) {
            const float ev = es[o][k];
            acc[o][0] = fmaf(ev, wv.x, acc[o][0]);
            acc[o][1] = fmaf(ev, wv.y, acc[o][1]);
            acc[o][2] = fmaf(ev, wv.z, acc[o][2]);
            acc[o][3] = fmaf(ev, wv.w, acc[o][3]);
        }
    }
    for (int o = 0; o < kHeadObj; ++o)
        if (o0 + o < n_obj)
            *(float4 *)&logits[(int64_t)(o0 + o) * NB + b] =
                make_float4(acc[o][0], acc[o][1], acc[o][2], acc[o][3]);
}

// Softmax cross-entropy per object (one wavefront each): loss_o and
// dlogits = (softmax - onehot) / n_obj.  Objects with a nonzero status or a
// label outside [0, 1024) contribute nothing.
__global__ __launch_bounds__(256) void ce_kernel(const float *__restrict__ logits,
                                                 const int32_t *__restrict__ labels,
                                                 const int32_t *__restrict__ status, int n_obj,
                                                 float *__restrict__ dlog,
                                                 float *__restrict__ loss_o) {
    const int lane = threadIdx.x % kWave;
    const int o = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (o >= n_obj) return;
    const float *z = logits + (int64_t)o * NB;
    float *d = dlog + (int64_t)o * NB;
    const int lab = labels[o];
    if (status[o] != 0 || lab < 0 || lab >= NB) {
        for (int b = lane; b < NB; b += kWave) d[b] = 0.0f;
        if (lane == 0) loss_o[o] = 0.0f;
        return;
    }
    float m = -__builtin_inff();
    for (int b = lane; b < NB; b += kWave) m = fmaxf(m, z[b]);
    m = (float)wave_max((double)m);
    float s = 0.0f;
    for (int b = lane; b < NB; b += kWave) s += __expf(z[b] - m);
    s = (float)wave_sum((double)s);
    const float lse = logf(s);
    const float inv_b = 1.0f / (float)n_obj;
    for (int b = lane; b < NB; b += kWave)
        d[b] = (__expf(z[b] - m - lse) - (b == lab ? 1.0f : 0.0f)) * inv_b;
    if (lane == 0) loss_o[o] = lse - (z[lab] - m);
}

// dW3[k][b] = sum_o emb[o][k] dlog[o][b] and db3[b] = sum_o dlog[o][b]:
// thread per bin, 16 k per workgroup row.
__global__ __launch_bounds__(256) void head_wgrad_kernel(const float *__restrict__ emb,
                                                         const float *__restrict__ dlog,
                                                         int n_obj, float *__restrict__ grad) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    const int k0 = blockIdx.y * 16;
    __shared__ float es[64][16];
    float acc[16] = {};
    float db = 0.0f;
    for (int o0 = 0; o0 < n_obj; o0 += 64) {
        __syncthreads();
        for (int i = threadIdx.x; i < 64 * 16; i += blockDim.x) {
            const int o = o0 + i / 16;
            es[i / 16][i % 16] = o < n_obj ? emb[(int64_t)o * H2 + k0 + i % 16] : 0.0f;
        }
        __syncthreads();
        const int oe = min(64, n_obj - o0);
        for (int oo = 0; oo < oe; ++oo) {
            const float dv = dlog[(int64_t)(o0 + oo) * NB + b];
            db += dv;
#pragma unroll
            for (int kk = 0; kk < 16; ++kk) acc[kk] = fmaf(es[oo][kk], dv, acc[kk]);
        }
    }
    for (int kk = 0; kk < 16; ++kk) grad[OFF_W3 + (k0 + kk) * NB + b] = acc[kk];
    if (blockIdx.y == 0) grad[OFF_B3 + b] = db;
}

// dE[o][k] = sum_b dlog[o][b] W3[k][b]: thread per k, 16 objects per workgroup.
__global__ __launch_bounds__(128) void head_dgrad_kernel(const float *__restrict__ dlog,
                                                         const float *__restrict__ prm,
                                                         int n_obj, float *__restrict__ dE) {
    const int k = threadIdx.x;
    const int o0 = blockIdx.x * 16;
    __shared__ float ds[16][64];
    float acc[16] = {};
    for (int b0 = 0; b0 < NB; b0 += 64) {
        __syncthreads();
        for (int i = threadIdx.x; i < 16 * 64; i += blockDim.x) {
            const int o = o0 + i / 64;
            ds[i / 64][i % 64] = o < n_obj ? dlog[(int64_t)o * NB + b0 + i % 64] : 0.0f;
        }
        __syncthreads();
        for (int bb = 0; bb < 64; ++bb) {
            const float wv = prm[OFF_W3 + k * NB + b0 + bb];
#pragma unroll
            for (int oo = 0; oo < 16; ++oo) acc[oo] = fmaf(ds[oo][bb], wv, acc[oo]);
        }
    }
    for (int oo = 0; oo < 16; ++oo)
        if (o0 + oo < n_obj) dE[(int64_t)(o0 + oo) * H2 + k] = acc[oo];
}

// Sums the per-wave W1/W2 partials, forms db2[u] = sum_o dE[o][u] act[o][u]
// (the mean-pool's gradient summed over each object's active points), and
// the mean loss.  Fixed summation order: deterministic.
__global__ __launch_bounds__(256) void grad_reduce_kernel(const float *__restrict__ partial,
                                                          int n_waves,
                                                          const float *__restrict__ dE,
                                                          const float *__restrict__ act,
                                                          const float *__restrict__ loss_o,
                                                          int n_obj, float *__restrict__ grad,
                                                          float *__restrict__ loss) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < kMlpGrad) {
        float s = 0.0f;
        for (int w = 0; w < n_waves; ++w) s += partial[(int64_t)w * kMlpGrad + j];
        grad[j] = s;  // W1 then W2: the same order as the parameter vector
    } else if (j < kMlpGrad + H2) {
        const int u = j - kMlpGrad;
        float s = 0.0f;
        for (int o = 0; o < n_obj; ++o) s += dE[(int64_t)o * H2 + u] * act[(int64_t)o * H2 + u];
        grad[OFF_B2 + u] = s;
    } else if (j == kMlpGrad + H2) {
        float s = 0.0f;
        for (int o = 0; o < n_obj; ++o) s += loss_o[o];
        *loss = n_obj > 0 ? s / (float)n_obj : 0.0f;
    }
}

// Adam on FP32 master weights (bias-corrected moments).
__global__ __launch_bounds__(256) void adam_kernel(float *__restrict__ p,
                                                   const float *__restrict__ gr,
                                                   float *__restrict__ m, float *__restrict__ v,
                                                   int64_t n, float lr, float b1, float b2,
                                                   float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = gr[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// Refine planning, one wavefront per object: the top_k largest bin values
// v_b = logit_b + gamma * score_b (either term absent when its pointer is
// null; NaN ranks lowest; lowest bin first among equal values), each widened
// by `margin` bins on both sides, merged into runs of consecutive bins, and
// each run turned into fine-grid index ranges [bin_k[first], bin_k[last + 1])
// cut into pieces of at most `chunk` frequencies.  Objects with fewer than
// full_below points get the whole grid instead.  Writes n_rng ranges per
// object (unused entries empty).
__global__ __launch_bounds__(256) void plan_kernel(const float *__restrict__ logits,
                                                   const float *__restrict__ scores, float gamma,
                                                   const int32_t *__restrict__ status,
                                                   const int64_t *__restrict__ offsets,
                                                   int full_below,
                                                   const int64_t *__restrict__ bin_k, int n_obj,
                                                   int top_k, int margin, int chunk, int n_rng,
                                                   int64_t *__restrict__ ranges) {
    const int lane = threadIdx.x % kWave;
    const int o = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (o >= n_obj) return;
    int64_t *rg = ranges + (int64_t)o * n_rng * 2;
    constexpr int PER = NB / kWave;  // bins b = lane * PER + j
    float z[PER];
    uint32_t sel = 0u;  // bit j: bin lane * PER + j selected (after widening)
    const bool whole = status[o] == 0 && offsets[o + 1] - offsets[o] < (int64_t)full_below;
    if (whole) sel = 0xffffu;
    if (status[o] == 0 && !whole) {
        for (int j = 0; j < PER; ++j) {
            const int64_t q = (int64_t)o * NB + lane * PER + j;
            float v = logits ? logits[q] : 0.0f;
            if (scores) v = fmaf(gamma, scores[q], v);
            z[j] = __builtin_isnan(v) ? -__builtin_inff() : v;
        }
        uint32_t taken = 0u;
        for (int r = 0; r < top_k; ++r) {
            float bv = -__builtin_inff();
            int bj = -1;
            for (int j = 0; j < PER; ++j)
                if (!((taken >> j) & 1u) && (bj < 0 || z[j] > bv)) {
                    bv = z[j];
                    bj = j;
                }
            // wave argmax: largest value, then lowest bin
            int key_b = bj < 0 ? 0x7fffffff : lane * PER + bj;
            float key_v = bj < 0 ? -__builtin_inff() : bv;
            for (int off = 1; off < kWave; off <<= 1) {
                const float ov = __shfl_xor(key_v, off);
                const int ob = __shfl_xor(key_b, off);
                if (ov > key_v || (ov == key_v && ob < key_b)) {
                    key_v = ov;
                    key_b = ob;
                }
            }
            if (key_b == 0x7fffffff) break;
            if (key_b / PER == lane) taken |= 1u << (key_b % PER);
            for (int j = 0; j < PER; ++j) {
                const int b = lane * PER + j;
                if (b >= key_b - margin && b <= key_b + margin) sel |= 1u << j;
            }
        }
    }
    // Serial scan by lane 0 over the selection bitmap (1024 bits).
    __shared__ uint32_t bits[4][kWave];
    const int wv = threadIdx.x / kWave;
    bits[wv][lane] = sel;
    wave_lds_sync();
    if (lane == 0) {
        int r = 0;
        int b = 0;
        while (b < NB && r < n_rng) {
            if (!((bits[wv][b / PER] >> (b % PER)) & 1u)) {
                ++b;
                continue;
            }
            int e = b;
            while (e + 1 < NB && ((bits[wv][(e + 1) / PER] >> ((e + 1) % PER)) & 1u)) ++e;
            int64_t k0 = bin_k[b];
            const int64_t k1 = bin_k[e + 1];
            while (k0 < k1 && r < n_rng) {
                const int64_t k2 = (k1 - k0 > chunk) ? k0 + chunk : k1;
                rg[2 * r] = k0;
                rg[2 * r + 1] = k2;
                ++r;
                k0 = k2;
            }
            b = e + 1;
        }
        for (; r < n_rng; ++r) {
            rg[2 * r] = 0;
            rg[2 * r + 1] = 0;
        }
    }
}

}  // namespace

int enc_fwd_lds_bytes() { return kW1f * 16 + kW2f * 16 + H2 * 4; }
int enc_bwd_lds_bytes(int waves) {
    return kW1f * 16 + kW2f * 16 + H2 * 4 + kW2b * 16 + waves * H2 * 4 + waves * kRowsT * kPT * 2;
}
int enc_mlp_grad_floats() { return kMlpGrad; }

hipError_t launch_enc_fwd(const EncArgs &A, int n_cu, hipStream_t s) {
    if (A.n_obj <= 0) return hipSuccess;
    const void *fn = (const void *)enc_fwd_kernel;
    const int bytes = enc_fwd_lds_bytes();
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, 256, (size_t)bytes);
    if (e != hipSuccess) return e;
    int64_t grid = (int64_t)std::max(per_cu, 1) * n_cu;
    grid = std::min<int64_t>(grid, (A.n_obj + 3) / 4);
    hipLaunchKernelGGL(enc_fwd_kernel, dim3((unsigned)grid), dim3(256), (size_t)bytes, s, A);
    return hipGetLastError();
}

int enc_bwd_waves(int n_obj, int n_cu) {
    return (int)std::min<int64_t>((int64_t)n_cu * 4, std::max<int64_t>(2, (n_obj + 1) / 2 * 2));
}

hipError_t launch_enc_bwd(const EncArgs &A, int n_waves, hipStream_t s) {
    const void *fn = (const void *)enc_bwd_kernel;
    const int bytes = enc_bwd_lds_bytes(2);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(enc_bwd_kernel, dim3((unsigned)(n_waves / 2)), dim3(128), (size_t)bytes, s,
                       A);
    return hipGetLastError();
}

hipError_t launch_head_fwd(const float *emb, const float *prm, int n_obj, float *logits,
                           hipStream_t s) {
    if (n_obj <= 0) return hipSuccess;
    hipLaunchKernelGGL(head_fwd_kernel, dim3((unsigned)((n_obj + kHeadObj - 1) / kHeadObj)),
                       dim3(256), 0, s, emb, prm, n_obj, logits);
    return hipGetLastError();
}

hipError_t launch_train_tail(const EncArgs &A, const float *logits, const int32_t *labels,
                             float *dlog, float *loss_o, float *dE, float *grad, float *loss,
                             int n_waves, hipStream_t s) {
    const int n = A.n_obj;
    hipLaunchKernelGGL(ce_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, logits, labels,
                       A.status, n, dlog, loss_o);
    hipLaunchKernelGGL(head_wgrad_kernel, dim3(NB / 256, H2 / 16), dim3(256), 0, s, A.emb, dlog, n,
                       grad);
    hipLaunchKernelGGL(head_dgrad_kernel, dim3((unsigned)((n + 15) / 16)), dim3(128), 0, s, dlog,
                       A.params, n, dE);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    EncArgs B = A;
    B.dE = dE;
    e = launch_enc_bwd(B, n_waves, s);
    if (e != hipSuccess) return e;
    const int total = kMlpGrad + H2 + 1;
    hipLaunchKernelGGL(grad_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s,
                       A.partial, n_waves, dE, A.act, loss_o, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_adam(float *p, const float *g, float *m, float *v, int64_t n, float lr,
                       float b1, float b2, float eps, float c1, float c2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(adam_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, g, m, v,
                       n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_plan(const float *logits, const float *scores, float gamma,
                       const int32_t *status, const int64_t *offsets, int full_below,
                       const int64_t *bin_k, int n_obj, int top_k, int margin, int chunk,
                       int n_rng, int64_t *ranges, hipStream_t s) {
    if (n_obj <= 0) return hipSuccess;
    hipLaunchKernelGGL(plan_kernel, dim3((unsigned)((n_obj + 3) / 4)), dim3(256), 0, s, logits,
                       scores, gamma, status, offsets, full_below, bin_k, n_obj, top_k, margin,
                       chunk, n_rng, ranges);
    return hipGetLastError();
}

}  // namespace ssg
