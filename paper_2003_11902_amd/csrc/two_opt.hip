// 2-opt on every ant's tour with neighbour lists and don't-look bits
// (Sec. 5.7, after Bentley): one workgroup per ant, tour, position, edge
// lengths and don't-look bits in LDS.
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
// a city without a move gets its bit set. Several cities are evaluated per
// round (see k_two_opt), which changes the speed and not the result.
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

__device__ __forceinline__ int64_t dd(const int32_t* dist, int n, uint32_t x, uint32_t y) {
    return (int64_t)dist[(size_t)x * n + y];
}

constexpr int kMaxWaves = 16;
constexpr int kMaxList = 512;  // cities examined per round (1024 threads / groups of >= 2)

struct Cand {
    int key;                 // (list index << 6) | lane in group
    int a, a1, c, c1;
    int i, j;                // cyclic position range to reverse
    int dac, da1c1;          // lengths of the two new edges
    int flags;               // bits 0-3: don't-look bit of a, a1, c, c1 before the round;
                             // bit 4: the edge left of position i becomes {a, c}
};

__device__ __forceinline__ uint32_t dlb_bit(const uint32_t* dlb, int x) { return (dlb[x >> 5] >> (x & 31)) & 1u; }

// The next `count` active cities (don't-look bit clear) from city a0,
// cyclically, into `list`; one wave. Entries in order: the word of a0 from
// bit a0&31, the following words, the word of a0 below bit a0&31; 64 words a
// pass, until `count` cities are listed.
__device__ void list_active(const uint32_t* dlb, int words, uint32_t lastmask, int a0, int count, uint16_t* list,
                            int lane) {
    const int w0 = a0 >> 5, b0 = a0 & 31;
    int found = 0;
    for (int base = 0; base <= words && found < count; base += kWave) {
        const int e = base + lane;
        uint32_t bits = 0u;
        int w = 0;
        if (e <= words) {
            uint32_t m;
            if (e == 0) {
                w = w0;
                m = 0xFFFFFFFFu << b0;
            } else if (e < words) {
                w = w0 + e;
                if (w >= words) w -= words;
                m = 0xFFFFFFFFu;
            } else {
                w = w0;
                m = b0 ? ((1u << b0) - 1u) : 0u;
            }
            if (w == words - 1) m &= lastmask;
            bits = ~dlb[w] & m;
        }
        const int cnt = __popc(bits);
        const int incl = wave_incl_scan(cnt, lane);
        int idx = found + incl - cnt;
        while (bits && idx < count) {
            list[idx++] = (uint16_t)(w * 32 + __ffs(bits) - 1);
            bits &= bits - 1u;
        }
        found += __builtin_amdgcn_readlane(incl, 63);
    }
}

// The 2-opt of one ant per workgroup. kLen: the tour's edge lengths are kept
// in LDS by position (len[p] = d(tour[p], tour[p+1])), so a move evaluation
// reads one distance from HBM instead of three.
//
// A round examines the next C active cities in cyclic index order (C =
// threads / group, a group of 2k lanes per city) against the current tour.
// The first of them (in that order) with an improving move is the city the
// sequential search reaches next with a move: the cities before it have none
// and get their bits set, its move is applied and it is examined again. With
// no move among the C, all C get their bits set. The number of active cities
// and the cursor are kept by every thread alike (no broadcast needed).
template <bool kLen>
__global__ __launch_bounds__(1024) void k_two_opt(Views vw, Shape s, const int32_t* __restrict__ nnd) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint16_t s_lists[2][kMaxList];  // by round parity
    __shared__ Cand s_cand[kMaxWaves];
    __shared__ int s_key[kMaxWaves];
    __shared__ unsigned long long s_len;
    const int n = s.n, k = s.ls_nn;
    const int ant = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int nthr = blockDim.x, nwaves = nthr >> 6;
    int gs = 1;
    while (gs < 2 * k) gs <<= 1;  // lanes per city (power of two <= 64)
    const int C = min(nthr / gs, kMaxList);
    uint16_t* tour = reinterpret_cast<uint16_t*>(smem);
    uint16_t* pos = tour + n;
    const size_t tp_bytes = (4 * (size_t)n + 15) & ~(size_t)15;
    int32_t* elen = reinterpret_cast<int32_t*>(smem + tp_bytes);
    uint32_t* dlb = reinterpret_cast<uint32_t*>(smem + tp_bytes + (kLen ? 4 * (size_t)n : 0));
    const int words = (n + 31) >> 5;
    const uint32_t lastmask = (n & 31) ? ((1u << (n & 31)) - 1u) : 0xFFFFFFFFu;
    const int32_t* dist = vw.dist;
    const uint16_t* nn = vw.lsnn;
    uint16_t* gtour = vw.tours + (size_t)ant * n;
    // after a failed construction the tour may not be a permutation
    if (vw.state->flags & 8u) return;

    for (int i = t; i < n; i += nthr) {
        const uint16_t v = gtour[i];
        tour[i] = v;
        pos[v] = (uint16_t)i;
    }
    for (int w = t; w < words; w += nthr) dlb[w] = 0u;
    if (t == 0) s_len = 0ull;
    __syncthreads();
    if (kLen)
        for (int i = t; i < n; i += nthr) elen[i] = dist[(size_t)tour[i] * n + tour[i + 1 == n ? 0 : i + 1]];

    int act = n, a0 = 0;  // active cities and cursor (the same in every thread)
    int ca = -1, cc = 0, cdac = 0;  // this lane's last (city, neighbour, distance) from the lists
    // every round sets a bit or shortens the tour; the cap only guards
    // against a search that would not end
    const long long max_rounds = 256ll * n + 4096;
    long long rounds = 0;
    if (wave == 0) list_active(dlb, words, lastmask, 0, min(C, n), s_lists[1], lane);
    while (act > 0) {
        if (++rounds > max_rounds) {
            if (t == 0) atomicOr(&vw.state->flags, 16u);
            return;
        }
        const int count = min(C, act);
        uint16_t* s_list = s_lists[rounds & 1];  // listed by wave 0 at the end of the last round

        __syncthreads();  // the list, the tour, positions, lengths and bits of this round

        // ---- evaluate every candidate move of the listed cities ----
        const int g = t / gs, rl = t % gs;
        bool ok = false;
        int a = 0, a1 = 0, c = 0, c1 = 0, dac = 0, da1c1 = 0, pa = 0, pc = 0;
        const bool pred_dir = rl >= k;
        if (g < count && rl < 2 * k) {
            a = s_list[g];
            const int r = pred_dir ? rl - k : rl;
            if (a != ca) {  // the list often starts where the last one did
                cc = nn[(size_t)a * k + r];
                cdac = nnd[(size_t)a * k + r];
                ca = a;
            }
            c = cc;
            dac = cdac;
            pa = pos[a];
            const int pa_n = pa + 1 == n ? 0 : pa + 1, pa_p = pa == 0 ? n - 1 : pa - 1;
            a1 = pred_dir ? tour[pa_p] : tour[pa_n];
            const int32_t daa1 = kLen ? elen[pred_dir ? pa_p : pa] : dist[(size_t)a * n + a1];
            const int64_t g1 = (int64_t)daa1 - dac;
            if (g1 > 0) {
                pc = pos[c];
                const int pc_n = pc + 1 == n ? 0 : pc + 1, pc_p = pc == 0 ? n - 1 : pc - 1;
                c1 = pred_dir ? tour[pc_p] : tour[pc_n];
                if (c != a1 && c1 != a) {
                    const int32_t dcc1 = kLen ? elen[pred_dir ? pc_p : pc] : dist[(size_t)c * n + c1];
                    da1c1 = dist[(size_t)a1 * n + c1];
                    ok = g1 + (int64_t)dcc1 - (int64_t)da1c1 > 0;
                }
            }
        }
        const uint64_t mask = __ballot(ok);
        if (mask != 0ull) {
            const int m = __ffsll((unsigned long long)mask) - 1;  // lowest lane: first city, first move
            if (lane == m) {
                // the two paths the move may reverse (positions from pa and pc:
                // a1 and c1 sit next to a and c); the shorter one, the first on a tie
                const int pa_n = pa + 1 == n ? 0 : pa + 1, pa_p = pa == 0 ? n - 1 : pa - 1;
                const int pc_n = pc + 1 == n ? 0 : pc + 1, pc_p = pc == 0 ? n - 1 : pc - 1;
                int i1, j1, i2, j2;
                if (!pred_dir) {  // a -> a1 ... c -> c1: a1..c or c1..a
                    i1 = pa_n;
                    j1 = pc;
                    i2 = pc_n;
                    j2 = pa;
                } else {          // a1 -> a ... c1 -> c: a..c1 or c..a1
                    i1 = pa;
                    j1 = pc_p;
                    i2 = pc;
                    j2 = pa_p;
                }
                int len1 = j1 - i1;
                if (len1 < 0) len1 += n;
                len1 += 1;
                const bool first = len1 <= n - len1;
                const int i = first ? i1 : i2, j = first ? j1 : j2;
                const int x = tour[i == 0 ? n - 1 : i - 1];  // stays left of the reversed path
                const int fl = (int)dlb_bit(dlb, a) | ((int)dlb_bit(dlb, a1) << 1) | ((int)dlb_bit(dlb, c) << 2) |
                               ((int)dlb_bit(dlb, c1) << 3) | ((x == a || x == c) ? 16 : 0);
                s_cand[wave] = Cand{(g << 6) | rl, a, a1, c, c1, i, j, dac, da1c1, fl};
                s_key[wave] = (g << 6) | rl;
            }
        } else if (lane == 0) {
            s_key[wave] = 0x7FFFFFFF;
        }
        __syncthreads();
        // the first move over all waves: keys are (list index, lane), distinct
        const uint32_t kk = lane < nwaves ? (uint32_t)s_key[lane] : 0x7FFFFFFFu;
        const uint32_t kmin = wave_min_u32<2>(kk);  // lanes 0-31 (kMaxWaves <= 32)
        const int best = __ffsll((unsigned long long)__ballot(kk == kmin)) - 1;
        const bool moved = kmin != 0x7FFFFFFFu;
        Cand mv{};
        if (moved) mv = s_cand[best];
        const int gstar = moved ? (mv.key >> 6) : count;  // the listed cities before it have no move
        const int last = s_list[count - 1];
        int newact = act - gstar;
        const int ends[4] = {mv.a, mv.a1, mv.c, mv.c1};
        if (moved) {
            // an end point's bit is set after the listing if it was set before
            // the round or if it lies in the listed part before the move's city
            int span = mv.a - a0;
            if (span < 0) span += n;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                int de = ends[e] - a0;
                if (de < 0) de += n;
                const bool was = ((mv.flags >> e) & 1) || (e > 0 && de < span);
                newact += was ? 1 : 0;
            }
        }
        const int a0_next = moved ? mv.a : (last + 1 == n ? 0 : last + 1);
        // Wave 0 owns the don't-look bits: the listed cities before the move's
        // city get theirs set (except the move's end points, whose bits end
        // clear), the end points' are cleared, and the next round's cities
        // are listed while the other waves reverse the path.
        if (wave == 0) {
            for (int q = lane; q < gstar; q += kWave) {
                const int x = s_list[q];
                if (!moved || (x != mv.a1 && x != mv.c && x != mv.c1))
                    atomicOr(&dlb[x >> 5], 1u << (x & 31));
            }
            if (moved && lane < 4 && ((mv.flags >> lane) & 1))
                atomicAnd(&dlb[ends[lane] >> 5], ~(1u << (ends[lane] & 31)));
            if (newact > 0)
                list_active(dlb, words, lastmask, a0_next, min(C, newact), s_lists[(rounds + 1) & 1], lane);
        }
        if (moved && (wave > 0 || nwaves == 1)) {
            // reverse positions i..j of the tour and i..j-1 of the edge lengths:
            // pair q swaps tour[i+q] and tour[j-q], and elen[i+q] and
            // elen[j-1-q] (for even lengths the middle pair of the lengths is
            // one cell swapped with itself)
            const int rt = nwaves == 1 ? t : t - kWave, rthr = nwaves == 1 ? nthr : nthr - kWave;
            int len = mv.j - mv.i;
            if (len < 0) len += n;
            len += 1;
            const int half = len / 2;
            for (int q = rt; q < half; q += rthr) {
                int p = mv.i + q;
                if (p >= n) p -= n;
                int r = mv.j - q;
                if (r < 0) r += n;
                int r1 = r - 1;
                if (r1 < 0) r1 += n;
                const uint16_t tp = tour[p], tr = tour[r];
                int32_t ep = 0, er = 0;
                if (kLen) {
                    ep = elen[p];
                    er = elen[r1];
                }
                tour[p] = tr;
                tour[r] = tp;
                pos[tr] = (uint16_t)p;
                pos[tp] = (uint16_t)r;
                if (kLen) {
                    elen[p] = er;
                    elen[r1] = ep;
                }
            }
            if (kLen && rt == 0) {  // the two new edges close the reversed path
                const int pl = mv.i == 0 ? n - 1 : mv.i - 1;
                const bool left_ac = (mv.flags >> 4) & 1;
                elen[pl] = left_ac ? mv.dac : mv.da1c1;
                elen[mv.j] = left_ac ? mv.da1c1 : mv.dac;
            }
        }
        a0 = a0_next;
        act = newact;
    }
    __syncthreads();
    // write back; the tour length from the final edges
    int64_t tl = 0;
    for (int i = t; i < n; i += nthr) {
        const uint16_t v = tour[i];
        gtour[i] = v;
        tl += kLen ? (int64_t)elen[i] : (int64_t)dist[(size_t)v * n + tour[i + 1 == n ? 0 : i + 1]];
    }
    tl = wave_sum_i64(tl);
    if (lane == 0) atomicAdd(&s_len, (unsigned long long)tl);
    __syncthreads();
    if (t == 0) vw.lengths[ant] = (int64_t)s_len;
}

// d(i, nn[i][r]) for the 2-opt neighbour lists
__global__ __launch_bounds__(256) void k_nn_dist(const int32_t* __restrict__ dist, const uint16_t* __restrict__ nn,
                                                 int n, int k, int32_t* __restrict__ out) {
    const size_t total = (size_t)n * k;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x)
        out[e] = dist[(e / k) * n + nn[e]];
}

}  // namespace

// dynamic LDS of the 2-opt kernel: tour and position (uint16), the edge
// lengths (int32) when `with_len`, and the don't-look bits
size_t two_opt_lds_bytes(const Shape& s, bool with_len) {
    return (size_t)((4 * s.n + 15) & ~15) + (with_len ? 4 * (size_t)s.n : 0) + 4 * (size_t)((s.n + 31) / 32);
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
    const bool with_len = two_opt_lds_bytes(s, true) + kTwoOptStaticLds <= (size_t)max_lds_per_block();
    const size_t lds = two_opt_lds_bytes(s, with_len);
    const void* kern = with_len ? (const void*)k_two_opt<true> : (const void*)k_two_opt<false>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    Views vv = v;
    Shape ss = s;
    void* args[] = {(void*)&vv, (void*)&ss, (void*)&nnd};
    return hipLaunchKernel(kern, dim3(s.ants), dim3(64 * s.two_opt_waves), args, lds, st);
}

}  // namespace mmas
