// Learned heuristic (a project addition beside the paper's eta = 1/d of
// Sec. 2.1): k-nearest-neighbour edge features, a 8 -> 128 -> 128 -> 1 GELU
// edge-scoring MLP in bfloat16 on MFMA with FP32 accumulation (inference,
// and training by binary cross-entropy with logits and Adam), and the
// installation eta_ij = (1/d_ij) * 2 sigmoid(s_ij) on the 16 nearest cities
// of i; the other edges of i take the multiplier of i's lowest score, so
// s = 0 gives the plain heuristic exactly.
//
// MFMA: v_mfma_f32_16x16x16_bf16. With lane l, row block q = l / 16 and
// column c = l % 16: the A operand of lane l is A[c][4q .. 4q+3] (row c,
// four consecutive k), the B operand is B[4q .. 4q+3][c] (column c), and the
// result holds D[4q + t][c], t = 0..3.
#include <cmath>
#include <cstddef>
#include <mutex>

#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

constexpr int kHid = 128;
constexpr int kIn = 16;
constexpr int kK = 16;  // nearest neighbours per city

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// nearest bfloat16, ties to even (finite inputs)
__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t b = __float_as_uint(x);
    b = b + 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// exp in FP32: clamp to [-104, 89], k = rint(x log2 e), r = x - k ln2 (ln2 as
// a 15-bit head and a rounded tail), exp(r) by its Taylor series through r^8,
// times 2^k.
__device__ __forceinline__ float exp_f32(float x) {
    const float kLog2e = __uint_as_float(0x3FB8AA3Bu);
    const float kLn2Hi = __uint_as_float(0x3F317200u);
    const float kLn2Lo = __uint_as_float(0x35BFBE8Eu);
    x = x > 89.0f ? 89.0f : x;
    x = x < -104.0f ? -104.0f : x;
    const float kf = __builtin_rintf(x * kLog2e);
    const float r = (x - kf * kLn2Hi) - kf * kLn2Lo;
    float p = 1.0f / 40320.0f;
    p = 1.0f / 5040.0f + r * p;
    p = 1.0f / 720.0f + r * p;
    p = 1.0f / 120.0f + r * p;
    p = 1.0f / 24.0f + r * p;
    p = 1.0f / 6.0f + r * p;
    p = 0.5f + r * p;
    p = 1.0f + r * p;
    p = 1.0f + r * p;
    return ldexpf(p, (int)kf);
}

__device__ __forceinline__ float sigmoid_f32(float s) { return 1.0f / (1.0f + exp_f32(-s)); }

// erf by Abramowitz and Stegun 7.1.26 (absolute error below 1.5e-7):
// erf(x) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-x^2),
// t = 1 / (1 + p x), x >= 0; odd in x.
__device__ __forceinline__ float erf_as(float x) {
    const float ax = fabsf(x);
    const float t = 1.0f / (1.0f + 0.3275911f * ax);
    const float poly =
        t * (0.254829592f + t * (-0.284496736f + t * (1.421413741f + t * (-1.453152027f + t * 1.061405429f))));
    const float y = 1.0f - poly * exp_f32(-ax * ax);
    return x < 0.0f ? -y : y;
}

// GELU(z) = z Phi(z) and its derivative Phi(z) + z phi(z)
__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erf_as(z * 0.70710678f)); }
__device__ __forceinline__ float gelu_d(float z) {
    return 0.5f * (1.0f + erf_as(z * 0.70710678f)) + z * 0.39894228f * exp_f32(-0.5f * z * z);
}

// ---- features ----------------------------------------------------------------

// in-degree counters cleared by a kernel rather than a memset node, so that
// the feature pass can be captured into a graph and replayed
__global__ __launch_bounds__(256) void k_zero_i32(int* __restrict__ a, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = 0;
}

__global__ __launch_bounds__(256) void k_feat_city(const int32_t* __restrict__ dist, const uint16_t* __restrict__ knn,
                                                   int n, float* __restrict__ dbar, int* __restrict__ indeg) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float s = 0.0f;
    for (int r = 0; r < kK; ++r) s = s + (float)dist[(size_t)i * n + knn[i * kK + r]];
    dbar[i] = s / 16.0f;
    for (int r = 0; r < kK; ++r) atomicAdd(&indeg[knn[i * kK + r]], 1);
}

// one thread per directed edge e = 16 i + r; FP32 features in the order of
// operations the oracle uses, then the bfloat16 MLP input row (8 features,
// 8 zeros)
__global__ __launch_bounds__(256) void k_feat_edge(const int32_t* __restrict__ dist, const float* __restrict__ xy,
                                                   const uint16_t* __restrict__ knn, const float* __restrict__ dbar,
                                                   const int* __restrict__ indeg, int n, float* __restrict__ feat,
                                                   uint16_t* __restrict__ X) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kK) return;
    const int i = e / kK, r = e % kK;
    const int j = knn[e];
    int back = 16;
    for (int t = 0; t < kK; ++t)
        if (knn[j * kK + t] == i) {
            back = t;
            break;
        }
    float f[8];
    f[0] = (float)dist[(size_t)i * n + j] / dbar[i];
    f[1] = (float)r / 15.0f;
    f[2] = (float)back / 16.0f;
    f[3] = (xy[2 * j] - xy[2 * i]) / dbar[i];
    f[4] = (xy[2 * j + 1] - xy[2 * i + 1]) / dbar[i];
    f[5] = (float)indeg[j] / 16.0f;
    f[6] = (float)indeg[i] / 16.0f;
    f[7] = dbar[j] / dbar[i];
    for (int c = 0; c < 8; ++c) {
        if (feat) feat[(size_t)e * 8 + c] = f[c];
        X[(size_t)e * kIn + c] = to_bf16(f[c]);
        X[(size_t)e * kIn + 8 + c] = 0;
    }
}

// ---- parameters ------------------------------------------------------------------
// FP32 master layout: W1 [16][128] | b1 [128] | W2 [128][128] | b2 [128] | w3 [128] | b3

constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kIn * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid;
constexpr int kParams = kOffB3 + 1;

// bfloat16 working copies: W1t [128 out][16 in], W2t [128 out][128 in],
// W2n [128 in][128 out], w3 [128]
constexpr int kPkW1t = 0;
constexpr int kPkW2t = kPkW1t + kHid * kIn;
constexpr int kPkW2n = kPkW2t + kHid * kHid;
constexpr int kPkW3 = kPkW2n + kHid * kHid;
constexpr int kPacked = kPkW3 + kHid;

__global__ __launch_bounds__(256) void k_pack(const float* __restrict__ p, uint16_t* __restrict__ pk) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < kHid * kHid; t += gridDim.x * blockDim.x) {
        const int a = t / kHid, b = t % kHid;          // W2[a][b], a = in, b = out
        pk[kPkW2n + a * kHid + b] = to_bf16(p[kOffW2 + a * kHid + b]);
        pk[kPkW2t + b * kHid + a] = to_bf16(p[kOffW2 + a * kHid + b]);
        if (t < kIn * kHid) {
            const int k = t / kHid, c = t % kHid;      // W1[k][c]
            pk[kPkW1t + c * kIn + k] = to_bf16(p[kOffW1 + k * kHid + c]);
        }
        if (t < kHid) pk[kPkW3 + t] = to_bf16(p[kOffW3 + t]);
    }
}

// ---- forward / backward tiles -------------------------------------------------------

// (the forward kernel allocates only the part before w2n: 55 KB, two
// workgroups per CU; the fused training kernel all of it)
struct Smem {
    uint16_t w1t[kHid * kIn];
    uint16_t w2t[kHid * kHid];
    uint16_t w3[kHid];
    float b1[kHid], b2[kHid];
    uint16_t x[64 * kIn];     // tile of 64 edges
    uint16_t h1[64 * kHid];
    uint16_t w2n[kHid * kHid];
    uint16_t dz2[64 * kHid];
    uint16_t dz1[64 * kHid];
    float red[4][3 * kHid + 2];
};
constexpr size_t kForwardSmem = offsetof(Smem, w2n);

__device__ void load_weights(Smem& sm, const float* __restrict__ p, const uint16_t* __restrict__ pk, bool need_w2n) {
    for (int t = threadIdx.x; t < kHid * kIn; t += blockDim.x) sm.w1t[t] = pk[kPkW1t + t];
    for (int t = threadIdx.x; t < kHid * kHid; t += blockDim.x) {
        sm.w2t[t] = pk[kPkW2t + t];
        if (need_w2n) sm.w2n[t] = pk[kPkW2n + t];
    }
    for (int t = threadIdx.x; t < kHid; t += blockDim.x) {
        sm.w3[t] = pk[kPkW3 + t];
        sm.b1[t] = p[kOffB1 + t];
        sm.b2[t] = p[kOffB2 + t];
    }
}

// four consecutive bfloat16 values at p (8-byte aligned) as an MFMA operand
__device__ __forceinline__ bf16x4 ld4(const uint16_t* p) { return *reinterpret_cast<const bf16x4*>(p); }

__device__ __forceinline__ bf16x4 gather4(const uint16_t* p, int stride) {
    bf16x4 v;
    v[0] = (short)p[0];
    v[1] = (short)p[stride];
    v[2] = (short)p[2 * stride];
    v[3] = (short)p[3 * stride];
    return v;
}

// Forward of the 16 edges rows0 .. rows0 + 15 of the tile held by this wave
// (X rows already in sm.x). Leaves Z1, Z2 (pre-activation, FP32, result
// layout) in z1 / z2, H1 (bfloat16) in sm.h1 and returns the partial score
// sum of this lane's rows 4q + t over its columns (reduce over c).
__device__ void forward16(Smem& sm, int rows0, int lane, float z1[8][4], float z2[8][4], float h2[8][4],
                          float spart[4]) {
    const int q = lane >> 4, c = lane & 15;
    const bf16x4 a1 = ld4(&sm.x[(rows0 + c) * kIn + 4 * q]);
    for (int nt = 0; nt < 8; ++nt) {
        const int col = nt * 16 + c;
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        d = mfma16(a1, ld4(&sm.w1t[col * kIn + 4 * q]), d);
        for (int t = 0; t < 4; ++t) {
            const float z = d[t] + sm.b1[col];
            z1[nt][t] = z;
            sm.h1[(rows0 + 4 * q + t) * kHid + col] = to_bf16(gelu(z));
        }
    }
    for (int t = 0; t < 4; ++t) spart[t] = 0.0f;
    for (int nt = 0; nt < 8; ++nt) {
        const int col = nt * 16 + c;
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
        for (int kt = 0; kt < 8; ++kt) {
            const bf16x4 a = ld4(&sm.h1[(rows0 + c) * kHid + kt * 16 + 4 * q]);
            const bf16x4 b = ld4(&sm.w2t[col * kHid + kt * 16 + 4 * q]);
            acc = mfma16(a, b, acc);
        }
        const float w3 = from_bf16(sm.w3[col]);
        for (int t = 0; t < 4; ++t) {
            const float z = acc[t] + sm.b2[col];
            z2[nt][t] = z;
            const float h = from_bf16(to_bf16(gelu(z)));
            h2[nt][t] = h;
            spart[t] += h * w3;
        }
    }
}

// sum over the 16 lanes that share q (xor over the low four lane bits)
__device__ __forceinline__ float sum16(float x) {
    for (int o = 1; o < 16; o <<= 1) x += __shfl_xor(x, o);
    return x;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const uint16_t* __restrict__ X, const float* __restrict__ p,
                                                     const uint16_t* __restrict__ pk, int64_t E,
                                                     float* __restrict__ s_out) {
    extern __shared__ __align__(16) uint8_t raw[];
    Smem& sm = *reinterpret_cast<Smem*>(raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    load_weights(sm, p, pk, false);
    const float b3 = p[kOffB3];
    const int64_t tiles = (E + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t e0 = tile * 64;
        __syncthreads();
        for (int t = threadIdx.x; t < 64 * kIn; t += blockDim.x) {
            const int64_t e = e0 + t / kIn;
            sm.x[t] = e < E ? X[e * kIn + t % kIn] : (uint16_t)0;
        }
        __syncthreads();
        float z1[8][4], z2[8][4], h2[8][4], sp[4];
        forward16(sm, wave * 16, lane, z1, z2, h2, sp);
        const int q = lane >> 4, c = lane & 15;
        for (int t = 0; t < 4; ++t) {
            const float s = sum16(sp[t]) + b3;
            const int64_t e = e0 + wave * 16 + 4 * q + t;
            if (c == 0 && e < E) s_out[e] = s;
        }
    }
}

// Fused forward and backward over tiles of 64 edges; each workgroup keeps its
// gradient sums in registers and writes them once to partial[blockIdx.x]
// (kParams floats) plus its loss sum to partial[gridDim.x * kParams + b].
__global__ __launch_bounds__(256) void k_mlp_train(const uint16_t* __restrict__ X, const float* __restrict__ f,
                                                   const float* __restrict__ p, const uint16_t* __restrict__ pk,
                                                   int64_t E, float* __restrict__ partial) {
    extern __shared__ __align__(16) uint8_t raw[];
    Smem& sm = *reinterpret_cast<Smem*>(raw);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = lane >> 4, c = lane & 15;
    load_weights(sm, p, pk, true);
    const float b3 = p[kOffB3];
    const float invE = 1.0f / (float)E;
    // gradient accumulators (result layout of the MFMA tiles this wave owns)
    f32x4 gw2[8][2];   // dW2 rows (in) 16 mt + ..., columns (out) 32 wave + 16 nt2 + c
    f32x4 gw1[2];      // dW1 rows (in) 0..15, columns 32 wave + 16 nt2 + c
    for (int mt = 0; mt < 8; ++mt)
        for (int u = 0; u < 2; ++u) gw2[mt][u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    gw1[0] = gw1[1] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    float gb1[8], gb2[8], gw3[8], gb3 = 0.0f, loss = 0.0f;
    for (int nt = 0; nt < 8; ++nt) gb1[nt] = gb2[nt] = gw3[nt] = 0.0f;

    const int64_t tiles = (E + 63) / 64;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t e0 = tile * 64;
        __syncthreads();
        for (int t = threadIdx.x; t < 64 * kIn; t += blockDim.x) {
            const int64_t e = e0 + t / kIn;
            sm.x[t] = e < E ? X[e * kIn + t % kIn] : (uint16_t)0;
        }
        __syncthreads();
        const int rows0 = wave * 16;
        float z1[8][4], z2[8][4], h2[8][4], sp[4];
        forward16(sm, rows0, lane, z1, z2, h2, sp);
        // dL/ds per row (zero past E)
        float g[4];
        for (int t = 0; t < 4; ++t) {
            const float s = sum16(sp[t]) + b3;
            const int64_t e = e0 + rows0 + 4 * q + t;
            g[t] = 0.0f;
            if (e < E) {
                const float fe = f[e];
                g[t] = (sigmoid_f32(s) - fe) * invE;
                if (c == 0) {
                    const float sp_ = s > 0.0f ? s + log1pf(exp_f32(-s)) : log1pf(exp_f32(s));
                    loss += sp_ - fe * s;
                }
            }
            if (c == 0) gb3 += g[t];
        }
        for (int nt = 0; nt < 8; ++nt) {
            const int col = nt * 16 + c;
            const float w3 = from_bf16(sm.w3[col]);
            for (int t = 0; t < 4; ++t) {
                gw3[nt] += h2[nt][t] * g[t];
                const uint16_t dz = to_bf16(g[t] * w3 * gelu_d(z2[nt][t]));
                gb2[nt] += from_bf16(dz);
                sm.dz2[(rows0 + 4 * q + t) * kHid + col] = dz;
            }
        }
        // dH1 = dZ2 W2^T for this wave's rows, then dZ1
        for (int nt = 0; nt < 8; ++nt) {
            const int col = nt * 16 + c;  // input unit of layer 2
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
            for (int kt = 0; kt < 8; ++kt) {
                const bf16x4 a = ld4(&sm.dz2[(rows0 + c) * kHid + kt * 16 + 4 * q]);
                const bf16x4 b = ld4(&sm.w2n[col * kHid + kt * 16 + 4 * q]);
                acc = mfma16(a, b, acc);
            }
            for (int t = 0; t < 4; ++t) {
                const uint16_t dz = to_bf16(acc[t] * gelu_d(z1[nt][t]));
                gb1[nt] += from_bf16(dz);
                sm.dz1[(rows0 + 4 * q + t) * kHid + col] = dz;
            }
        }
        __syncthreads();
        // dW2 += H1^T dZ2 and dW1 += X^T dZ1 over the 64 edges; this wave owns
        // output columns 32 wave .. 32 wave + 31
        for (int kk = 0; kk < 4; ++kk) {
            const int er = kk * 16 + 4 * q;  // edge rows of this lane's operand
            for (int u = 0; u < 2; ++u) {
                const int ocol = wave * 32 + u * 16 + c;
                const bf16x4 bz2 = gather4(&sm.dz2[er * kHid + ocol], kHid);
                const bf16x4 bz1 = gather4(&sm.dz1[er * kHid + ocol], kHid);
                for (int mt = 0; mt < 8; ++mt) {
                    const bf16x4 a = gather4(&sm.h1[er * kHid + mt * 16 + c], kHid);
                    gw2[mt][u] = mfma16(a, bz2, gw2[mt][u]);
                }
                const bf16x4 ax = gather4(&sm.x[er * kIn + c], kIn);
                gw1[u] = mfma16(ax, bz1, gw1[u]);
            }
        }
    }
    // write this workgroup's partial sums
    float* out = partial + (size_t)blockIdx.x * kParams;
    for (int mt = 0; mt < 8; ++mt)
        for (int u = 0; u < 2; ++u)
            for (int t = 0; t < 4; ++t)
                out[kOffW2 + (mt * 16 + 4 * q + t) * kHid + wave * 32 + u * 16 + c] = gw2[mt][u][t];
    for (int u = 0; u < 2; ++u)
        for (int t = 0; t < 4; ++t) out[kOffW1 + (4 * q + t) * kHid + wave * 32 + u * 16 + c] = gw1[u][t];
    // column sums: over the four row blocks q of the wave, then over the waves
    for (int nt = 0; nt < 8; ++nt) {
        float a = gb1[nt], b = gb2[nt], w = gw3[nt];
        a += __shfl_xor(a, 16);
        a += __shfl_xor(a, 32);
        b += __shfl_xor(b, 16);
        b += __shfl_xor(b, 32);
        w += __shfl_xor(w, 16);
        w += __shfl_xor(w, 32);
        if (q == 0) {
            sm.red[wave][nt * 16 + c] = a;
            sm.red[wave][kHid + nt * 16 + c] = b;
            sm.red[wave][2 * kHid + nt * 16 + c] = w;
        }
    }
    float lb = gb3, ll = loss;
    for (int o = 1; o < 64; o <<= 1) {
        lb += __shfl_xor(lb, o);
        ll += __shfl_xor(ll, o);
    }
    if (lane == 0) {
        sm.red[wave][3 * kHid] = lb;
        sm.red[wave][3 * kHid + 1] = ll;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < 3 * kHid + 2; t += blockDim.x) {
        const float v = ((sm.red[0][t] + sm.red[1][t]) + sm.red[2][t]) + sm.red[3][t];
        if (t < kHid) out[kOffB1 + t] = v;
        else if (t < 2 * kHid) out[kOffB2 + t - kHid] = v;
        else if (t < 3 * kHid) out[kOffW3 + t - 2 * kHid] = v;
        else if (t == 3 * kHid) out[kOffB3] = v;
        else partial[(size_t)gridDim.x * kParams + blockIdx.x] = v;
    }
}

// grad[i] = sum over workgroups of partial[w][i], in workgroup order; the loss
// sum goes to grad[kParams]
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ partial, int groups,
                                                     float* __restrict__ grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i > kParams) return;
    float s = 0.0f;
    if (i < kParams)
        for (int w = 0; w < groups; ++w) s += partial[(size_t)w * kParams + i];
    else
        for (int w = 0; w < groups; ++w) s += partial[(size_t)groups * kParams + w];
    grad[i] = s;
}

// Adam in FP32: m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g g;
// p -= lr (m / c1) / (sqrt(v / c2) + eps)
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                              float* __restrict__ v, int count, float lr, float b1, float b2, float eps,
                                              float c1, float c2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float o1 = 1.0f - b1, o2 = 1.0f - b2;
    const float gi = g[i];
    const float mi = b1 * m[i] + o1 * gi;
    const float vi = b2 * v[i] + o2 * (gi * gi);
    m[i] = mi;
    v[i] = vi;
    p[i] = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// eta_ij = fl(fl(1/d_ij) * fl(2 sigma(s_ij))) on the 16 nearest of i, 1/d
// elsewhere; heur = eta^beta. Dense: heur is n*n. Candidate-only trails:
// heur is n*cl along the candidate lists.
__global__ __launch_bounds__(256) void k_install(const int32_t* __restrict__ dist, const uint16_t* __restrict__ knn,
                                                 const float* __restrict__ s, const uint16_t* __restrict__ cand, int n,
                                                 int cl, int beta, int dense, float* __restrict__ heur) {
    const size_t total = dense ? (size_t)n * n : (size_t)n * cl;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
        const int i = dense ? (int)(e / n) : (int)(e / cl);
        const int j = dense ? (int)(e % n) : (int)cand[e];
        float h = 0.0f;
        if (i != j) {
            const float eta = 1.0f / (float)dist[(size_t)i * n + j];
            // own score if j is among the 16 nearest, else the lowest score of i
            float smin = s[i * kK], sc = 0.0f;
            bool found = false;
            for (int r = 0; r < kK; ++r) {
                const float v = s[i * kK + r];
                smin = v < smin ? v : smin;
                if (!found && knn[i * kK + r] == j) {
                    sc = v;
                    found = true;
                }
            }
            const float x = eta * (2.0f * sigmoid_f32(found ? sc : smin));
            h = powi(x, beta);
        }
        heur[e] = h;
    }
}

// target of edge (i, knn[i][r]): the share of the R tours that use it
__global__ __launch_bounds__(256) void k_labels(const uint16_t* __restrict__ tours, int R, int n,
                                                const uint16_t* __restrict__ knn, float* __restrict__ label) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * kK) return;
    const int i = e / kK, j = knn[e];
    int hits = 0;
    for (int t = 0; t < R; ++t) {
        const uint16_t* tr = tours + (size_t)t * n;
        // positions of i and j: scan (n is small in training instances)
        int pi = -1, pj = -1;
        for (int k = 0; k < n; ++k) {
            if (tr[k] == i) pi = k;
            if (tr[k] == j) pj = k;
        }
        const int dpos = pi > pj ? pi - pj : pj - pi;
        hits += (dpos == 1 || dpos == n - 1) ? 1 : 0;
    }
    label[e] = (float)hits / (float)R;
}

int grid_of(size_t total) {
    size_t g = (total + 255) / 256;
    if (g > 65536) g = 65536;
    return g < 1 ? 1 : (int)g;
}

}  // namespace

int mlp_param_count() { return kParams; }
int mlp_packed_count() { return kPacked; }

hipError_t launch_features(const int32_t* dist, const float* xy, const uint16_t* knn, int n, float* dbar, int* indeg,
                           float* feat, uint16_t* X, hipStream_t st) {
    k_zero_i32<<<(n + 255) / 256, 256, 0, st>>>(indeg, n);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_feat_city<<<(n + 255) / 256, 256, 0, st>>>(dist, knn, n, dbar, indeg);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_feat_edge<<<(n * kK + 255) / 256, 256, 0, st>>>(dist, xy, knn, dbar, indeg, n, feat, X);
    return hipGetLastError();
}

hipError_t launch_pack(const float* p, uint16_t* pk, hipStream_t st) {
    k_pack<<<64, 256, 0, st>>>(p, pk);
    return hipGetLastError();
}

static hipError_t smem_attr(const void* k, size_t bytes) {
    return hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_mlp_forward(const uint16_t* X, const float* p, const uint16_t* pk, int64_t E, float* s,
                              hipStream_t st) {
    hipError_t e = smem_attr((const void*)k_mlp_forward, kForwardSmem);
    if (e != hipSuccess) return e;
    const int64_t tiles = (E + 63) / 64;
    const int grid = (int)(tiles < 2048 ? tiles : 2048);
    k_mlp_forward<<<grid < 1 ? 1 : grid, 256, kForwardSmem, st>>>(X, p, pk, E, s);
    return hipGetLastError();
}

hipError_t launch_mlp_train(const uint16_t* X, const float* f, const float* p, const uint16_t* pk, int64_t E,
                            float* partial, int groups, float* grad, hipStream_t st) {
    hipError_t e = smem_attr((const void*)k_mlp_train, sizeof(Smem));
    if (e != hipSuccess) return e;
    k_mlp_train<<<groups, 256, sizeof(Smem), st>>>(X, f, p, pk, E, partial);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_grad_reduce<<<(kParams + 1 + 255) / 256, 256, 0, st>>>(partial, groups, grad);
    return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, float lr, float b1, float b2, float eps, float c1,
                       float c2, hipStream_t st) {
    k_adam<<<(kParams + 255) / 256, 256, 0, st>>>(p, g, m, v, kParams, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t launch_install(const int32_t* dist, const uint16_t* knn, const float* s, const uint16_t* cand, int n, int cl,
                          int beta, int dense, float* heur, hipStream_t st) {
    const size_t total = dense ? (size_t)n * n : (size_t)n * cl;
    k_install<<<grid_of(total), 256, 0, st>>>(dist, knn, s, cand, n, cl, beta, dense, heur);
    return hipGetLastError();
}

hipError_t launch_labels(const uint16_t* tours, int R, int n, const uint16_t* knn, float* label, hipStream_t st) {
    k_labels<<<(n * kK + 255) / 256, 256, 0, st>>>(tours, R, n, knn, label);
    return hipGetLastError();
}

}  // namespace mmas

// ---- scratch for callers that cannot allocate ------------------------------------

// The feature pass's per-city scratch (dbar as FP32, then the in-degree
// counters as int32: 8 bytes per city) for the largest instance the library
// takes, held by every GPU the library runs on until the process ends. Host
// code never passes this name to a kernel (on the host it is only a stand-in
// for the symbol): it uses the device address hipGetSymbolAddress returns.
constexpr int kScratchCities = 65535;
static __device__ __align__(256) uint8_t scratch[8 * (size_t)kScratchCities];

namespace {
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kScratchDevices];  // device address of `scratch`, per device

// The current device's copy of `scratch`, looked up on the first call on
// that device (with it current) and kept.
mmas_status scratch_of_current_device(void** out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return mmas::hip_fail(e, "hipGetDevice (static feature scratch)");
    if (dev < 0 || dev >= kScratchDevices) return MMAS_EUNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return mmas::hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                           "hipGetSymbolAddress (static feature scratch)");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MMAS_OK;
}
}  // namespace

// ---- C ABI ----------------------------------------------------------------------

namespace {
hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }
mmas_status st_of(hipError_t e) { return e == hipSuccess ? MMAS_OK : mmas::hip_fail(e, "learned-heuristic kernel"); }
}  // namespace

extern "C" {

int32_t mmas_mlp_param_count(void) { return mmas::mlp_param_count(); }
int32_t mmas_mlp_packed_count(void) { return mmas::mlp_packed_count(); }

mmas_status mmas_mlp_features(const int32_t* dist_dev, const float* xy_dev, int32_t n, void* scratch_dev,
                              uint16_t* knn_dev, float* feat_dev, uint16_t* x_dev, void* hip_stream) {
    if (!dist_dev || !xy_dev || !scratch_dev || !knn_dev || !x_dev || n < 17 || n > 65535) return MMAS_EINVAL;
    hipStream_t st = as_stream(hip_stream);
    hipError_t e = mmas::launch_nearest(dist_dev, n, 16, knn_dev, st);
    if (e != hipSuccess) return st_of(e);
    float* dbar = reinterpret_cast<float*>(scratch_dev);
    int* indeg = reinterpret_cast<int*>(dbar + n);
    return st_of(mmas::launch_features(dist_dev, xy_dev, knn_dev, n, dbar, indeg, feat_dev, x_dev, st));
}

mmas_status mmas_mlp_features_noalloc(const int32_t* dist_dev, const float* xy_dev, int32_t n, uint16_t* knn_dev,
                                      float* feat_dev, uint16_t* x_dev, void* hip_stream) {
    if (!dist_dev || !xy_dev || !knn_dev || !x_dev || n < 17) return MMAS_EINVAL;
    if (n > kScratchCities) return MMAS_EINVAL;  // beyond the static scratch (and the library's n)
    void* ws = nullptr;
    const mmas_status got = scratch_of_current_device(&ws);
    if (got != MMAS_OK) return got;
    hipStream_t st = as_stream(hip_stream);
    hipError_t e = mmas::launch_nearest(dist_dev, n, 16, knn_dev, st);
    if (e != hipSuccess) return st_of(e);
    // the in-degree counters are cleared by a kernel inside launch_features
    float* dbar = reinterpret_cast<float*>(ws);
    int* indeg = reinterpret_cast<int*>(dbar + n);
    return st_of(mmas::launch_features(dist_dev, xy_dev, knn_dev, n, dbar, indeg, feat_dev, x_dev, st));
}

mmas_status mmas_mlp_pack(const float* params_dev, uint16_t* packed_dev, void* hip_stream) {
    if (!params_dev || !packed_dev) return MMAS_EINVAL;
    return st_of(mmas::launch_pack(params_dev, packed_dev, as_stream(hip_stream)));
}

mmas_status mmas_mlp_forward(const uint16_t* x_dev, int64_t edges, const float* params_dev, const uint16_t* packed_dev,
                             float* s_dev, void* hip_stream) {
    if (edges < 0 || (edges > 0 && (!x_dev || !params_dev || !packed_dev || !s_dev))) return MMAS_EINVAL;
    if (edges == 0) return MMAS_OK;
    return st_of(mmas::launch_mlp_forward(x_dev, params_dev, packed_dev, edges, s_dev, as_stream(hip_stream)));
}

mmas_status mmas_mlp_grad(const uint16_t* x_dev, const float* target_dev, int64_t edges, const float* params_dev,
                          const uint16_t* packed_dev, float* partial_dev, int32_t groups, float* grad_dev,
                          void* hip_stream) {
    if (edges < 1 || groups < 1 || groups > 4096 || !x_dev || !target_dev || !params_dev || !packed_dev ||
        !partial_dev || !grad_dev)
        return MMAS_EINVAL;
    return st_of(mmas::launch_mlp_train(x_dev, target_dev, params_dev, packed_dev, edges, partial_dev, groups,
                                        grad_dev, as_stream(hip_stream)));
}

mmas_status mmas_mlp_adam(float* params_dev, const float* grad_dev, float* m_dev, float* v_dev, float lr, float beta1,
                          float beta2, float eps, int32_t step, void* hip_stream) {
    if (!params_dev || !grad_dev || !m_dev || !v_dev || step < 1) return MMAS_EINVAL;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
    return st_of(mmas::launch_adam(params_dev, grad_dev, m_dev, v_dev, lr, beta1, beta2, eps, c1, c2,
                                   as_stream(hip_stream)));
}

mmas_status mmas_mlp_labels(const uint16_t* tours_dev, int32_t tours, int32_t n, const uint16_t* knn_dev,
                            float* target_dev, void* hip_stream) {
    if (!tours_dev || !knn_dev || !target_dev || tours < 1 || n < 17) return MMAS_EINVAL;
    return st_of(mmas::launch_labels(tours_dev, tours, n, knn_dev, target_dev, as_stream(hip_stream)));
}

}  // extern "C"
