// Set-up kernels (Alg. 1 before its main loop): validation of the distance
// matrix, eta^beta, candidate and neighbour lists, the nearest-neighbour tour,
// the initial trail limits and tau <- tau_max.
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

// flags: 1 = asymmetric, 2 = non-zero diagonal, 4 = non-positive off-diagonal.
// 32x32 tiles; the transposed tile is staged in LDS so both reads coalesce.
// With `directed` (ATSP) an asymmetric matrix is valid and flag 1 is not set.
__global__ __launch_bounds__(256) void k_validate(const int32_t* __restrict__ d, int n, int directed,
                                                  uint32_t* __restrict__ flags) {
    __shared__ int32_t tile[32][33];
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;
    for (int j = ty; j < 32; j += 8) {
        const int r = by + j, c = bx + tx;
        if (r < n && c < n) tile[j][tx] = d[(size_t)r * n + c];
    }
    __syncthreads();
    uint32_t f = 0;
    for (int j = ty; j < 32; j += 8) {
        const int r = bx + j, c = by + tx;  // element d[r][c]; tile holds d[by+.][bx+.]
        if (r < n && c < n) {
            const int32_t x = d[(size_t)r * n + c];
            const int32_t y = tile[tx][j];  // d[c][r]
            if (x != y && !directed) f |= 1u;
            if (r == c) {
                if (x != 0) f |= 2u;
            } else if (x <= 0) {
                f |= 4u;
            }
        }
    }
    if (f) atomicOr(flags, f);
}

__global__ __launch_bounds__(256) void k_heur_dense(const int32_t* __restrict__ d, int n, int beta,
                                                    float* __restrict__ heur) {
    const size_t total = (size_t)n * n;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / n), j = (int)(e % n);
        heur[e] = (i == j) ? 0.0f : heur_from_dist(d[e], beta);
    }
}

__global__ __launch_bounds__(256) void k_heur_cand(const int32_t* __restrict__ d, const uint16_t* __restrict__ cand,
                                                   int n, int cl, int beta, float* __restrict__ heur) {
    const size_t total = (size_t)n * cl;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const size_t i = e / cl;
        heur[e] = heur_from_dist(d[i * n + cand[e]], beta);
    }
}

// Row i: the k nearest other cities by (distance, index). Round r takes the
// smallest (d, j) strictly above the one taken in round r-1.
__global__ __launch_bounds__(256) void k_nearest(const int32_t* __restrict__ d, int n, int k,
                                                 uint16_t* __restrict__ out) {
    __shared__ uint64_t part[4];
    const int i = blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t* row = d + (size_t)i * n;
    uint64_t prev = 0;  // keys are (d << 32 | j) with d >= 1 for j != i
    for (int r = 0; r < k; ++r) {
        uint64_t best = ~0ull;
        for (int j = threadIdx.x; j < n; j += 256) {
            if (j == i) continue;
            const uint64_t key = ((uint64_t)(uint32_t)row[j] << 32) | (uint32_t)j;
            if (key > prev && key < best) best = key;
        }
        best = wave_min_u64(best);
        if (lane == 0) part[wave] = best;
        __syncthreads();
        uint64_t m = part[0];
        for (int w = 1; w < 4; ++w) m = part[w] < m ? part[w] : m;
        __syncthreads();
        if (threadIdx.x == 0) out[(size_t)i * k + r] = (uint16_t)(m & 0xFFFFu);
        prev = m;
    }
}

// Nearest-neighbour tour from city 0 (one wave; visited bits in LDS), then
// its length. The candidate list is sorted by (d, index) and holds the cl
// nearest cities, so when one of them is unvisited the first such is the
// nearest unvisited city; only otherwise is the whole row scanned for the
// smallest (d, index).
__global__ __launch_bounds__(64) void k_nn_tour(const int32_t* __restrict__ d, const uint16_t* __restrict__ cand,
                                                int cl, int n, uint16_t* __restrict__ tour,
                                                mmas_device_state* __restrict__ st) {
    extern __shared__ uint32_t vis[];  // ceil(n/32) words
    const int lane = threadIdx.x;
    const int words = (n + 31) >> 5;
    for (int w = lane; w < words; w += kWave) vis[w] = 0u;
    if (lane == 0) vis[0] = 1u;
    int cur = 0;
    uint32_t tbuf = 0;       // lane (k & 63) holds the city of step k
    uint32_t prev_last = 0;  // last city of the previous 64-step chunk
    int64_t len = 0;
    for (int k = 1; k < n; ++k) {
        int nxt = -1;
        if (cl > 0) {
            const uint32_t c = cand[(size_t)cur * cl + (lane < cl ? lane : cl - 1)];
            const bool free = (lane < cl) & !((vis[c >> 5] >> (c & 31)) & 1u);
            const uint64_t m = __ballot(free);
            if (m) nxt = __builtin_amdgcn_readlane((int)c, __ffsll((unsigned long long)m) - 1);
        }
        if (nxt < 0) {
            const int32_t* row = d + (size_t)cur * n;
            uint64_t best = ~0ull;
            for (int j = lane; j < n; j += kWave) {
                const uint64_t key = ((uint64_t)(uint32_t)row[j] << 32) | (uint32_t)j;
                const bool seen = (vis[j >> 5] >> (j & 31)) & 1u;
                best = (!seen && key < best) ? key : best;
            }
            const uint64_t m = wave_min_u64(best);
            if (m == ~0ull) {  // no unvisited city: unreachable for k < n
                if (lane == 0) atomicOr(&st->flags, 8u);
                return;
            }
            nxt = (int)(m & 0xFFFFFFFFu);
        }
        if (lane == 0) vis[nxt >> 5] |= 1u << (nxt & 31);
        const int slot = k & 63;
        if (lane == slot) tbuf = (uint32_t)nxt;
        cur = nxt;
        if (slot == 63 || k == n - 1) {
            const int k0 = k - slot;
            const uint32_t prev = __shfl_up(tbuf, 1);
            if (lane <= slot) {
                tour[k0 + lane] = (uint16_t)tbuf;
                const uint32_t from = lane == 0 ? prev_last : prev;
                if (k0 + lane > 0) len += d[(size_t)from * n + tbuf];
            }
            prev_last = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, slot);
        }
    }
    if (lane == 0) {
        tour[0] = 0;
        len += d[(size_t)cur * n];  // closing edge back to city 0
    }
    len = wave_sum_i64(len);
    if (lane == 0) st->nn_len = len;
}

__global__ void k_init_state(mmas_device_state* st, float rho, int n, double pdec) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        float lo, hi;
        trail_limits(rho, st->nn_len, n, pdec, &lo, &hi);
        st->tau_min = lo;
        st->tau_max = hi;
        st->delta = 0.0f;
        st->ib_ant = -1;
        st->ib_len = -1;
        st->gb_len = -1;
        st->updates = 0u;
    }
}

__global__ __launch_bounds__(256) void k_fill_tau(float* __restrict__ tau, size_t count,
                                                  const mmas_device_state* __restrict__ st) {
    const float v = st->tau_max;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (size_t)gridDim.x * blockDim.x)
        tau[e] = v;
}

int grid_for(size_t total, int block) {
    size_t g = (total + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

hipError_t launch_validate(const Views& v, const Shape& s, hipStream_t st) {
    const int tiles = (s.n + 31) / 32;
    k_validate<<<dim3(tiles, tiles), dim3(32, 8), 0, st>>>(v.dist, s.n, s.directed, &v.state->flags);
    return hipGetLastError();
}

hipError_t launch_heuristic(const Views& v, const Shape& s, hipStream_t st) {
    if (s.pher == MMAS_PHER_DENSE) {
        const size_t total = (size_t)s.n * s.n;
        k_heur_dense<<<grid_for(total, 256), 256, 0, st>>>(v.dist, s.n, s.beta, v.heur);
    } else {
        const size_t total = (size_t)s.n * s.cl;
        k_heur_cand<<<grid_for(total, 256), 256, 0, st>>>(v.dist, v.cand, s.n, s.cl, s.beta, v.heur);
    }
    return hipGetLastError();
}

hipError_t launch_nearest(const int32_t* dist, int n, int k, uint16_t* out, hipStream_t st) {
    if (k <= 0) return hipSuccess;
    k_nearest<<<n, 256, 0, st>>>(dist, n, k, out);
    return hipGetLastError();
}

hipError_t launch_nn_tour(const Views& v, const Shape& s, hipStream_t st) {
    const size_t lds = sizeof(uint32_t) * (size_t)((s.n + 31) / 32);
    k_nn_tour<<<1, kWave, lds, st>>>(v.dist, v.cand, s.cl, s.n, v.nn_tour, v.state);
    return hipGetLastError();
}

hipError_t launch_init_trails(const Views& v, const Shape& s, hipStream_t st) {
    k_init_state<<<1, 64, 0, st>>>(v.state, s.rho, s.n, s.pdec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t count = s.pher == MMAS_PHER_DENSE ? (size_t)s.n * s.n : (size_t)s.n * s.cl;
    k_fill_tau<<<grid_for(count, 256), 256, 0, st>>>(v.tau, count, v.state);
    return hipGetLastError();
}

}  // namespace mmas
