// 2-opt on every ant's tour with neighbour lists and don't-look bits
// (Sec. 5.7, after Bentley), one wave64 per ant, tour and position arrays in
// LDS.
//
// The result is that of the sequential first-improvement search: cities are
// examined in index order, cyclically, skipping those whose don't-look bit is
// set, until every bit is set. For city a, the 2k candidate moves (successor
// direction then predecessor direction, neighbours by rank) are evaluated in
// parallel, one per lane; a move counts only while the first partial gain
// g1 = d(a, a') - d(a, c) is positive (it cannot grow with the rank, so this
// is the sequential "stop at the first g1 <= 0"); the lowest lane with a
// positive total gain is the move the sequential search would take. The move
// reverses the shorter of its two paths (the one starting next to a on a
// tie), its four end points get their bits cleared and a is examined again;
// a city without a move gets its bit set.
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

__device__ __forceinline__ int64_t dd(const int32_t* dist, int n, uint32_t x, uint32_t y) {
    return (int64_t)dist[(size_t)x * n + y];
}

// reverse the cyclic path of positions i..j (inclusive) in parallel
__device__ void reverse_path(uint16_t* tour, uint16_t* pos, int n, int i, int j, int lane) {
    const int len = ((j - i + n) % n) + 1;
    for (int t = lane; t < len / 2; t += kWave) {
        int p = i + t;
        if (p >= n) p -= n;
        int q = j - t;
        if (q < 0) q += n;
        const uint16_t tp = tour[p], tq = tour[q];
        tour[p] = tq;
        tour[q] = tp;
        pos[tq] = (uint16_t)p;
        pos[tp] = (uint16_t)q;
    }
}

// first city at or after `a` (cyclically) whose don't-look bit is clear;
// the caller guarantees one exists
__device__ int next_active(const uint32_t* dlb, int n, int a, int lane) {
    const int words = (n + 31) >> 5;
    const int w0 = a >> 5;
    const uint32_t first = ~dlb[w0] & (0xFFFFFFFFu << (a & 31));
    uint32_t lastmask = (n & 31) ? ((1u << (n & 31)) - 1u) : 0xFFFFFFFFu;
    if (w0 == words - 1) {
        const uint32_t f = first & lastmask;
        if (f) return w0 * 32 + __ffs(f) - 1;
    } else if (first) {
        return w0 * 32 + __ffs(first) - 1;
    }
    // the following words, cyclically (ending with w0 itself, whole)
    for (int base = 1; base <= words; base += kWave) {
        const int off = base + lane;
        uint32_t fr = 0u;
        if (off <= words) {
            const int w = (w0 + off) % words;
            fr = ~dlb[w];
            if (w == words - 1) fr &= lastmask;
        }
        const uint64_t m = __ballot(fr != 0u);
        if (m) {
            const int l = __ffsll((unsigned long long)m) - 1;
            const int w = (w0 + base + l) % words;
            const uint32_t f = (uint32_t)__builtin_amdgcn_readlane((int)fr, l);
            return w * 32 + __ffs(f) - 1;
        }
    }
    return a;  // not reached
}

__global__ __launch_bounds__(64) void k_two_opt(Views vw, Shape s, const int32_t* __restrict__ nnd) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int n = s.n, k = s.ls_nn;
    const int ant = blockIdx.x;
    const int lane = threadIdx.x;
    uint16_t* tour = reinterpret_cast<uint16_t*>(smem);
    uint16_t* pos = tour + n;
    uint32_t* dlb = reinterpret_cast<uint32_t*>(smem + ((4 * n + 15) & ~15));
    const int words = (n + 31) >> 5;
    const int32_t* dist = vw.dist;
    const uint16_t* nn = vw.lsnn;
    uint16_t* gtour = vw.tours + (size_t)ant * n;

    for (int i = lane; i < n; i += kWave) {
        const uint16_t t = gtour[i];
        tour[i] = t;
        pos[t] = (uint16_t)i;
    }
    for (int w = lane; w < words; w += kWave) dlb[w] = 0u;

    int active = n;  // cities whose bit is clear (uniform)
    int a = 0;
    while (active > 0) {
        a = next_active(dlb, n, a, lane);
        const int pa = pos[a];
        const uint32_t asucc = tour[pa + 1 == n ? 0 : pa + 1];
        const uint32_t apred = tour[pa == 0 ? n - 1 : pa - 1];
        // lane l < k: successor direction, rank l; k <= l < 2k: predecessor, rank l - k
        bool ok = false;
        uint32_t c = 0, c1 = 0, a1 = 0;
        const bool pred_dir = lane >= k;
        if (lane < 2 * k) {
            const int r = pred_dir ? lane - k : lane;
            a1 = pred_dir ? apred : asucc;
            c = nn[(size_t)a * k + r];
            const int64_t g1 = dd(dist, n, a, a1) - (int64_t)nnd[(size_t)a * k + r];
            if (g1 > 0) {
                const int pc = pos[c];
                c1 = pred_dir ? tour[pc == 0 ? n - 1 : pc - 1] : tour[pc + 1 == n ? 0 : pc + 1];
                if (c != a1 && c1 != (uint32_t)a) {
                    const int64_t gain = g1 + dd(dist, n, c, c1) - dd(dist, n, a1, c1);
                    ok = gain > 0;
                }
            }
        }
        const uint64_t mask = __ballot(ok);
        if (mask == 0ull) {
            if (lane == 0) dlb[a >> 5] |= 1u << (a & 31);
            active -= 1;
            a = a + 1 == n ? 0 : a + 1;
            continue;
        }
        const int m = __ffsll((unsigned long long)mask) - 1;
        const bool pdir = m >= k;
        const uint32_t mc = (uint32_t)__builtin_amdgcn_readlane((int)c, m);
        const uint32_t mc1 = (uint32_t)__builtin_amdgcn_readlane((int)c1, m);
        const uint32_t ma1 = pdir ? apred : asucc;
        int i1, j1, i2, j2;
        if (!pdir) {  // a -> a1 ... c -> c1: reverse a1..c or c1..a
            i1 = pos[ma1];
            j1 = pos[mc];
            i2 = pos[mc1];
            j2 = pa;
        } else {      // a1 -> a ... c1 -> c: reverse a..c1 or c..a1
            i1 = pa;
            j1 = pos[mc1];
            i2 = pos[mc];
            j2 = pos[ma1];
        }
        const int len1 = ((j1 - i1 + n) % n) + 1;
        if (len1 <= n - len1)
            reverse_path(tour, pos, n, i1, j1, lane);
        else
            reverse_path(tour, pos, n, i2, j2, lane);
        // clear the bits of the four end points (all lanes read, lane 0 writes)
        const uint32_t ends[4] = {(uint32_t)a, ma1, mc, mc1};
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t x = ends[e];
            const uint32_t bit = 1u << (x & 31);
            if (dlb[x >> 5] & bit) {
                active += 1;
                if (lane == 0) dlb[x >> 5] &= ~bit;
            }
        }
    }
    int64_t len = 0;
    for (int i = lane; i < n; i += kWave) {
        const uint16_t t = tour[i];
        gtour[i] = t;
        len += dd(dist, n, t, tour[i + 1 == n ? 0 : i + 1]);
    }
    len = wave_sum_i64(len);
    if (lane == 0) vw.lengths[ant] = len;
}

// d(i, nn[i][r]) for the 2-opt neighbour lists
__global__ __launch_bounds__(256) void k_nn_dist(const int32_t* __restrict__ dist, const uint16_t* __restrict__ nn,
                                                 int n, int k, int32_t* __restrict__ out) {
    const size_t total = (size_t)n * k;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
        out[e] = dist[(e / k) * n + nn[e]];
}

}  // namespace

size_t two_opt_lds_bytes(const Shape& s) {
    return (size_t)((4 * s.n + 15) & ~15) + 4 * (size_t)((s.n + 31) / 32);
}

hipError_t launch_two_opt_prepare(const Views& v, const Shape& s, int32_t* nnd, hipStream_t st) {
    if (s.ls_nn <= 0) return hipSuccess;
    const size_t total = (size_t)s.n * s.ls_nn;
    int g = (int)((total + 255) / 256);
    if (g > 65536) g = 65536;
    k_nn_dist<<<g, 256, 0, st>>>(v.dist, v.lsnn, s.n, s.ls_nn, nnd);
    return hipGetLastError();
}

hipError_t launch_two_opt(const Views& v, const Shape& s, const int32_t* nnd, hipStream_t st) {
    const size_t lds = two_opt_lds_bytes(s);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_two_opt, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    k_two_opt<<<s.ants, 64, lds, st>>>(v, s, nnd);
    return hipGetLastError();
}

}  // namespace mmas
