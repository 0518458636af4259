// Per-iteration kernels around construction (Alg. 1, Sec. 2.1):
//  - choice_info = tau^alpha * eta^beta, dense and along the candidate lists,
//    and its reciprocal beside both (Sec. 4.2.2: the reciprocal of every
//    weight computed once per iteration, so that a key is a product);
//  - the iteration best, the global best and the trail limits (one workgroup);
//  - evaporation, deposit on both directions of the iteration best's edges (on
//    (i, succ(i)) alone for the asymmetric TSP) and the [tau_min, tau_max] clamp, fused with the refresh of choice_info (the
//    paper's evaporation and deposition kernels in one pass; each entry is
//    independent, so no atomics are needed).
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

// dense: one workgroup per row
__global__ __launch_bounds__(256) void k_choice_dense(const float* __restrict__ tau, const float* __restrict__ heur,
                                                      const uint16_t* __restrict__ cand, int n, int cl, int alpha,
                                                      float* __restrict__ choice, float* __restrict__ choice_inv,
                                                      float* __restrict__ chc, float* __restrict__ chc_inv) {
    const size_t i = blockIdx.x;
    const float* trow = tau + i * n;
    const float* hrow = heur + i * n;
    float* crow = choice + i * n;
    float* irow = choice_inv + i * n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const float c = powi(trow[j], alpha) * hrow[j];
        crow[j] = c;
        irow[j] = 1.0f / c;
    }
    for (int r = threadIdx.x; r < cl; r += blockDim.x) {
        const int j = cand[i * cl + r];
        const float c = powi(trow[j], alpha) * hrow[j];
        chc[i * cl + r] = c;
        chc_inv[i * cl + r] = 1.0f / c;
    }
}

// candidate-only trails: heur is n*cl along the lists
__global__ __launch_bounds__(256) void k_choice_cand(const float* __restrict__ tau, const float* __restrict__ heur,
                                                     size_t count, int alpha, float* __restrict__ chc,
                                                     float* __restrict__ chc_inv) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        const float c = powi(tau[e], alpha) * heur[e];
        chc[e] = c;
        chc_inv[e] = 1.0f / c;
    }
}

// Iteration best = shortest tour, lowest ant on ties. If it beats the global
// best (or there is none yet), it becomes the global best and the limits are
// recomputed from its length. Then the successor and predecessor of every
// city along the tour that deposits: the iteration best, or the global best
// (Sec. 2.1 allows either). One workgroup of any size
// (a multiple of 64, at most 1024 threads).
__device__ void best_and_limits(const Views& vw, const Shape& s) {
    __shared__ int64_t plen[16];
    __shared__ int32_t pant[16];
    __shared__ int s_ib;
    __shared__ int s_improved;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int64_t blen = INT64_MAX;
    int32_t bant = INT32_MAX;
    for (int a = threadIdx.x; a < s.ants; a += blockDim.x) {
        const int64_t L = vw.lengths[a];
        if (L < blen) {  // ascending a: the first minimum is the lowest ant
            blen = L;
            bant = a;
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        const int64_t ol = __shfl_xor(blen, o);
        const int32_t oa = __shfl_xor(bant, o);
        if (ol < blen || (ol == blen && oa < bant)) {
            blen = ol;
            bant = oa;
        }
    }
    if (lane == 0) {
        plen[wave] = blen;
        pant[wave] = bant;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t L = plen[0];
        int32_t a = pant[0];
        for (int w = 1; w < nw; ++w)
            if (plen[w] < L || (plen[w] == L && pant[w] < a)) {
                L = plen[w];
                a = pant[w];
            }
        mmas_device_state* st = vw.state;
        st->ib_ant = a;
        st->ib_len = L;
        const int improved = (st->gb_len < 0 || L < st->gb_len) ? 1 : 0;
        if (improved) {
            st->gb_len = L;
            float lo, hi;
            trail_limits(s.rho, L, s.n, s.pdec, &lo, &hi);
            st->tau_min = lo;
            st->tau_max = hi;
        }
        st->delta = (float)(1.0 / (double)(s.deposit == MMAS_DEPOSIT_GLOBAL_BEST ? st->gb_len : L));
        st->updates += 1u;
        s_ib = a;
        s_improved = improved;
    }
    __syncthreads();
    const uint16_t* t = vw.tours + (size_t)s_ib * s.n;
    const int n = s.n;
    if (s.deposit == MMAS_DEPOSIT_GLOBAL_BEST && !s_improved) {
        // the global best deposits and is unchanged: its stored tour
        for (int k = threadIdx.x; k < n; k += blockDim.x) {
            const uint16_t a = vw.gb_tour[k], b = vw.gb_tour[k + 1 == n ? 0 : k + 1];
            vw.succ[a] = b;
            vw.pred[b] = a;
        }
        return;
    }
    for (int k = threadIdx.x; k < n; k += blockDim.x) {
        const uint16_t a = t[k], b = t[k + 1 == n ? 0 : k + 1];
        vw.succ[a] = b;
        vw.pred[b] = a;
        if (s_improved) vw.gb_tour[k] = a;
    }
}

__global__ __launch_bounds__(1024) void k_best(Views vw, Shape s) { best_and_limits(vw, s); }

__device__ __forceinline__ float evaporate_deposit(float t, bool dep, float keep, float tmin, float tmax,
                                                   float delta) {
    float v = keep * t;
    if (v < tmin) v = tmin;
    if (dep) v = v + delta;
    if (v > tmax) v = tmax;
    return v;
}

// dense: one workgroup per row i. The candidate entries of chc are computed
// first from the old trails (each thread recomputes its entry's new value),
// then the row is rewritten.
__device__ void update_dense_row(const Views& vw, const Shape& s, size_t i) {
    const int n = s.n, cl = s.cl;
    const mmas_device_state* st = vw.state;
    const float tmin = st->tau_min, tmax = st->tau_max, delta = st->delta;
    const float keep = 1.0f - s.rho;
    const int si = vw.succ[i], pi = s.directed ? -1 : (int)vw.pred[i];
    float* trow = vw.tau + i * n;
    const float* hrow = vw.heur + i * n;
    float* crow = vw.choice + i * n;
    float* irow = vw.choice_inv + i * n;
    for (int r = threadIdx.x; r < cl; r += blockDim.x) {
        const int j = vw.cand[i * cl + r];
        const float t = evaporate_deposit(trow[j], j == si || j == pi, keep, tmin, tmax, delta);
        const float c = powi(t, s.alpha) * hrow[j];
        vw.chc[i * cl + r] = c;
        vw.chc_inv[i * cl + r] = 1.0f / c;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        const float t = evaporate_deposit(trow[j], j == si || j == pi, keep, tmin, tmax, delta);
        trow[j] = t;
        const float c = powi(t, s.alpha) * hrow[j];
        crow[j] = c;
        irow[j] = 1.0f / c;
    }
}

// candidate-only trails, row i (its cl stored entries)
__device__ void update_cand_row(const Views& vw, const Shape& s, size_t i) {
    const mmas_device_state* st = vw.state;
    const float tmin = st->tau_min, tmax = st->tau_max, delta = st->delta;
    const float keep = 1.0f - s.rho;
    const int si = vw.succ[i], pi = s.directed ? -1 : (int)vw.pred[i];
    for (int r = threadIdx.x; r < s.cl; r += blockDim.x) {
        const size_t e = i * s.cl + r;
        const int j = vw.cand[e];
        const float t = evaporate_deposit(vw.tau[e], j == si || j == pi, keep, tmin, tmax, delta);
        vw.tau[e] = t;
        const float c = powi(t, s.alpha) * vw.heur[e];
        vw.chc[e] = c;
        vw.chc_inv[e] = 1.0f / c;
    }
}

__global__ __launch_bounds__(256) void k_update_dense(Views vw, Shape s) { update_dense_row(vw, s, blockIdx.x); }

// batches: one workgroup per instance for the best, then one per row
__global__ __launch_bounds__(1024) void k_batch_best(const BatchItem* __restrict__ items, uint32_t* it_dev,
                                                     uint32_t* queue) {
    best_and_limits(items[blockIdx.x].v, items[blockIdx.x].s);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *it_dev += 1u;  // construction of this iteration is done
        *queue = 0u;    // re-arm the tile queue for the next construction
    }
}

__global__ __launch_bounds__(256) void k_batch_update(const BatchItem* __restrict__ items, int count,
                                                      const int* __restrict__ row_start) {
    // instance of this row: last start <= blockIdx.x
    int lo = 0, hi = count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (row_start[mid] <= (int)blockIdx.x) lo = mid;
        else hi = mid - 1;
    }
    const Views vw = items[lo].v;
    const Shape s = items[lo].s;
    const size_t i = blockIdx.x - row_start[lo];
    if (s.pher == MMAS_PHER_DENSE)
        update_dense_row(vw, s, i);
    else
        update_cand_row(vw, s, i);
}

__global__ __launch_bounds__(256) void k_update_cand(Views vw, Shape s) {
    const size_t count = (size_t)s.n * s.cl;
    const mmas_device_state* st = vw.state;
    const float tmin = st->tau_min, tmax = st->tau_max, delta = st->delta;
    const float keep = 1.0f - s.rho;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / s.cl;
        const int j = vw.cand[e];
        const bool dep = j == vw.succ[i] || (!s.directed && j == vw.pred[i]);
        const float t = evaporate_deposit(vw.tau[e], dep, keep, tmin, tmax, delta);
        vw.tau[e] = t;
        const float c = powi(t, s.alpha) * vw.heur[e];
        vw.chc[e] = c;
        vw.chc_inv[e] = 1.0f / c;
    }
}

int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_choice(const Views& v, const Shape& s, hipStream_t st) {
    if (s.pher == MMAS_PHER_DENSE) {
        k_choice_dense<<<s.n, 256, 0, st>>>(v.tau, v.heur, v.cand, s.n, s.cl, s.alpha, v.choice, v.choice_inv, v.chc,
                                            v.chc_inv);
    } else {
        const size_t count = (size_t)s.n * s.cl;
        k_choice_cand<<<grid_for(count, 256), 256, 0, st>>>(v.tau, v.heur, count, s.alpha, v.chc, v.chc_inv);
    }
    return hipGetLastError();
}

hipError_t launch_batch_update(const BatchItem* items, int count, const int* row_start, int total_rows,
                               uint32_t* it_dev, uint32_t* queue, hipStream_t st) {
    k_batch_best<<<count, 256, 0, st>>>(items, it_dev, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_batch_update<<<total_rows, 256, 0, st>>>(items, count, row_start);
    return hipGetLastError();
}

hipError_t launch_update(const Views& v, const Shape& s, hipStream_t st) {
    k_best<<<1, 1024, 0, st>>>(v, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (s.pher == MMAS_PHER_DENSE) {
        k_update_dense<<<s.n, 256, 0, st>>>(v, s);
    } else {
        const size_t count = (size_t)s.n * s.cl;
        k_update_cand<<<grid_for(count, 256), 256, 0, st>>>(v, s);
    }
    return hipGetLastError();
}

}  // namespace mmas
