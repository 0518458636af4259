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

constexpr int kMaxWaves = 16;
constexpr int kListCap = 64;  // list entries kept, one per lane of the first wave

// A wave's first move: its end points, their positions, the new edges'
// lengths; flags bit 0 = predecessor direction, bits 1-3 = don't-look bits
// of a1, c, c1 before the round.
struct Move {
    int a, a1, c, c1;
    int pa, pc;
    int dac, da1c1;
    int flags;
};
constexpr uint32_t kNoMove = 0xFFFFFFFFu;

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
// A round examines the first E entries of a list of the next active cities
// in cyclic index order (E = threads / group, a group of 2k lanes per city,
// at most 64) against the current tour. The first of them (in that order)
// with an improving move is the city the sequential search reaches next with
// a move: the cities before it have none and get their bits set, its move is
// applied and it is examined again. Without a move all E get their bits set.
// Any prefix of the active cities in cyclic order from the cursor serves as
// the list, so the next list is the old one from the move's city (or from
// the first city not examined) on, with the end points that became active
// inside its range merged in; the don't-look bits are scanned again only
// when that list gets short. The first wave keeps the list (one entry per
// lane), the bits, the cursor and the count of active cities; the others
// reverse the path meanwhile.
template <bool kLen>
__global__ __launch_bounds__(1024) void k_two_opt(Views vw, Shape s, const int32_t* __restrict__ nnd) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ uint16_t s_lists[2][kListCap];  // by round parity
    __shared__ int s_count[2];                  // entries of each list (0: the search has ended)
    __shared__ uint32_t s_best[2];              // lowest thread (list index, lane in group) with a move
    __shared__ Move s_mv[kMaxWaves];            // each wave's first move
    __shared__ unsigned long long s_len;
    const int n = s.n, k = s.ls_nn;
    const int ant = blockIdx.x;
    const int t = threadIdx.x, lane = t & 63;
    // wave-uniform values are read into scalar registers (readfirstlane), so
    // that the bookkeeping of a round takes scalar branches
    const int wave = __builtin_amdgcn_readfirstlane(t >> 6);
    const int nthr = blockDim.x, nwaves = nthr >> 6;
    int gs = 1;
    while (gs < 2 * k) gs <<= 1;  // lanes per city (power of two <= 64)
    const int lg = __builtin_ctz(gs);
    const int E = min(nthr >> lg, kListCap);  // cities examined per round
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
    if (t == 0) {
        s_len = 0ull;
        s_best[0] = s_best[1] = kNoMove;
    }
    __syncthreads();
    if (kLen)
        for (int i = t; i < n; i += nthr) elen[i] = dist[(size_t)tour[i] * n + tour[i + 1 == n ? 0 : i + 1]];

    // Roles after a round's move is known: wave 0 sets and clears the
    // don't-look bits and tops the next list up from them, wave 1 merges the
    // next list from the current one, the other waves reverse the path (with
    // fewer waves, wave 0 also merges, and a single wave does everything).
    const int merge_wave = nwaves > 2 ? 1 : 0;
    const int rev_wave0 = nwaves > 2 ? 2 : nwaves - 1;
    int act = n, a0 = 0;            // active cities, cursor (kept alike by the first two waves)
    int ca = -1, cc = 0, cdac = 0;  // this lane's last (city, neighbour, distance) from the lists
    // a list shorter than this is topped up from the bits
    const int refill = min(E, 8);
    // every round sets a bit or shortens the tour; the cap only guards
    // against a search that would not end
    const long long max_rounds = 256ll * n + 4096;
    long long rounds = 0;
    if (wave == 0) {
        list_active(dlb, words, lastmask, 0, min(kListCap, n), s_lists[1], lane);
        if (lane == 0) s_count[1] = min(kListCap, n);
    }
    for (;;) {
        ++rounds;
        const int par = (int)(rounds & 1);
        const uint16_t* s_list = s_lists[par];

        __syncthreads();  // the list, the tour, positions, lengths and bits of this round
        // (the list entries are read beside the count: one LDS round trip)
        const int g = t >> lg, rl = t & (gs - 1);
        const int a_l = s_list[g < kListCap ? g : 0];
        const int le_l = s_list[lane];
        const int count = __builtin_amdgcn_readfirstlane(s_count[par]);
        if (count == 0) break;
        if (rounds > max_rounds) {
            if (t == 0) atomicOr(&vw.state->flags, 16u);
            return;
        }
        const int ev = min(count, E);
        const int le = lane < count ? le_l : 0;  // the list, one entry a lane (used by waves 0 and 1)

        // ---- evaluate every candidate move of the first ev listed cities ----
        const bool pred_dir = rl >= k;
        bool ok = false;
        int a = 0, a1 = 0, c = 0, c1 = 0, dac = 0, da1c1 = 0, pa = 0, pc = 0, fl = 0;
        if (g < ev && rl < 2 * k) {
            a = a_l;
            const int r = pred_dir ? rl - k : rl;
            if (a != ca) {  // the list often starts where the last one did
                cc = nn[(size_t)a * k + r];
                cdac = nnd[(size_t)a * k + r];
                ca = a;
            }
            c = cc;
            dac = cdac;
            // both ends' positions, then both tour neighbours and edge lengths
            pa = pos[a];
            pc = pos[c];
            const int pa_n = pa + 1 == n ? 0 : pa + 1, pa_p = pa == 0 ? n - 1 : pa - 1;
            const int pc_n = pc + 1 == n ? 0 : pc + 1, pc_p = pc == 0 ? n - 1 : pc - 1;
            a1 = tour[pred_dir ? pa_p : pa_n];
            c1 = tour[pred_dir ? pc_p : pc_n];
            const int64_t daa1 = kLen ? (int64_t)elen[pred_dir ? pa_p : pa] : (int64_t)dist[(size_t)a * n + a1];
            const int64_t g1 = daa1 - dac;
            if (g1 > 0 && c != a1 && c1 != a) {
                const int32_t dcc1 = kLen ? elen[pred_dir ? pc_p : pc] : dist[(size_t)c * n + c1];
                da1c1 = dist[(size_t)a1 * n + c1];
                // the end points' don't-look bits, read while the distance loads
                fl = (pred_dir ? 1 : 0) | ((int)dlb_bit(dlb, a1) << 1) | ((int)dlb_bit(dlb, c) << 2) |
                     ((int)dlb_bit(dlb, c1) << 3);
                ok = g1 + (int64_t)dcc1 - (int64_t)da1c1 > 0;
            }
        }
        const uint64_t mask = __ballot(ok);
        if (mask != 0ull && lane == __ffsll((unsigned long long)mask) - 1) {
            // lowest lane: first city, first move of this wave
            s_mv[wave] = Move{a, a1, c, c1, pa, pc, dac, da1c1, fl};
            atomicMin(&s_best[par], (uint32_t)t);  // thread index: list index, then lane in group
        }
        __syncthreads();
        // the first move over all waves
        const uint32_t best = __builtin_amdgcn_readfirstlane(s_best[par]);
        const bool moved = best != kNoMove;
        Move mv{};
        if (moved) {
            const Move m = s_mv[best >> 6];
            mv = Move{__builtin_amdgcn_readfirstlane(m.a),   __builtin_amdgcn_readfirstlane(m.a1),
                      __builtin_amdgcn_readfirstlane(m.c),   __builtin_amdgcn_readfirstlane(m.c1),
                      __builtin_amdgcn_readfirstlane(m.pa),  __builtin_amdgcn_readfirstlane(m.pc),
                      __builtin_amdgcn_readfirstlane(m.dac), __builtin_amdgcn_readfirstlane(m.da1c1),
                      __builtin_amdgcn_readfirstlane(m.flags)};
        }
        const int gstar = moved ? (int)(best >> lg) : ev;  // the listed cities before it have no move

        if (wave <= merge_wave) {
            const int last = __builtin_amdgcn_readlane(le, count - 1);
            auto cyc = [&](int x) { return x >= a0 ? x - a0 : x - a0 + n; };
            // The end points a1, c, c1: their don't-look bits before the
            // round (w), cyclic places (q), and the places of those merged
            // into the next list (inactive before, inside (a, last]; n for
            // the others). Everything here is wave-uniform but the lists.
            const int e1 = mv.a1, e2 = mv.c, e3 = mv.c1;
            const int w1 = (mv.flags >> 1) & 1, w2 = (mv.flags >> 2) & 1, w3 = (mv.flags >> 3) & 1;
            const int qa = cyc(mv.a), ql = cyc(last), q1 = cyc(e1), q2 = cyc(e2), q3 = cyc(e3);
            const int m1 = moved && w1 && q1 > qa && q1 <= ql ? q1 : n;
            const int m2 = moved && w2 && q2 > qa && q2 <= ql ? q2 : n;
            const int m3 = moved && w3 && q3 > qa && q3 <= ql ? q3 : n;
            // the listed cities before the move's city lose their bits (except
            // end points); the end points are all active afterwards: those
            // inactive before, and those listed before the move's city, count
            // again
            const int newact = act - gstar +
                               (moved ? (int)(w1 | (q1 < qa)) + (int)(w2 | (q2 < qa)) + (int)(w3 | (q3 < qa)) : 0);
            const int ee = lane == 0 ? e1 : lane == 1 ? e2 : e3;
            const int cap = min(kListCap, newact);
            // kept: the move's city (first) and the entries after it, or the
            // entries not examined; merged end points in cyclic order
            const int keep0 = moved ? gstar + 1 : gstar, head = moved ? 1 : 0;
            const int merged = (int)(m1 < n) + (int)(m2 < n) + (int)(m3 < n);
            int len = newact > 0 ? min(cap, head + count - keep0 + merged) : 0;
            uint16_t* nl = s_lists[par ^ 1];
            if (wave == 0) {
                if (lane == 0) s_best[par ^ 1] = kNoMove;  // for the next round
                const bool is_end = moved && (le == e1 || le == e2 || le == e3);
                if (lane < gstar && !is_end) atomicOr(&dlb[le >> 5], 1u << (le & 31));
                const int we = lane == 0 ? w1 : lane == 1 ? w2 : w3;
                if (moved && lane < 3 && we) atomicAnd(&dlb[ee >> 5], ~(1u << (ee & 31)));
            }
            if (wave == merge_wave && newact > 0) {
                const bool keep = lane >= keep0 && lane < count;
                const int cx = cyc(le);
                const int idx = head + lane - keep0 + (int)(m1 < cx) + (int)(m2 < cx) + (int)(m3 < cx);
                if (keep && idx < cap) nl[idx] = (uint16_t)le;
                // lanes 0-2: the place of merged end point e1, e2, e3 (lane 0
                // first writes the move's city)
                const int r1 = __popcll(__ballot(keep && cx < m1));
                const int r2 = __popcll(__ballot(keep && cx < m2));
                const int r3 = __popcll(__ballot(keep && cx < m3));
                const int mm = lane == 0 ? m1 : lane == 1 ? m2 : m3;
                const int rr = lane == 0 ? r1 : lane == 1 ? r2 : r3;
                const int ie = head + rr + (int)(m1 < mm) + (int)(m2 < mm) + (int)(m3 < mm);
                if (moved && lane == 0) nl[0] = (uint16_t)mv.a;
                if (lane < 3 && mm < n && ie < cap) nl[ie] = (uint16_t)ee;
            }
            int a0n = last + 1 == n ? 0 : last + 1;
            if (len > 0) a0n = moved ? mv.a : __builtin_amdgcn_readlane(le, gstar);
            if (len < cap && len < refill) {
                // the next active cities after the last listed one (after the
                // bits above: wave 0's own LDS operations complete in order)
                if (wave == 0)
                    list_active(dlb, words, lastmask, last + 1 == n ? 0 : last + 1, cap - len, nl + len, lane);
                len = cap;
            }
            if (wave == 0 && lane == 0) s_count[par ^ 1] = len;
            a0 = a0n;
            act = newact;
        }
        if (moved && wave >= rev_wave0) {
            // the two paths the move may reverse (a1 and c1 sit next to a and
            // c); the shorter one, the first on a tie
            const bool pd = mv.flags & 1;
            const int pa_n = mv.pa + 1 == n ? 0 : mv.pa + 1, pa_p = mv.pa == 0 ? n - 1 : mv.pa - 1;
            const int pc_n = mv.pc + 1 == n ? 0 : mv.pc + 1, pc_p = mv.pc == 0 ? n - 1 : mv.pc - 1;
            const int i1 = pd ? mv.pa : pa_n, j1 = pd ? pc_p : mv.pc;  // a1..c or a..c1
            const int i2 = pd ? mv.pc : pc_n, j2 = pd ? pa_p : mv.pa;  // c1..a or c..a1
            int len1 = j1 - i1;
            if (len1 < 0) len1 += n;
            len1 += 1;
            const bool first = len1 <= n - len1;
            const int mi = first ? i1 : i2, mj = first ? j1 : j2;
            // reverse positions i..j of the tour and i..j-1 of the edge lengths:
            // pair q swaps tour[i+q] and tour[j-q], and elen[i+q] and
            // elen[j-1-q] (for even lengths the middle pair of the lengths is
            // one cell swapped with itself)
            const int rt = t - rev_wave0 * kWave, rthr = nthr - rev_wave0 * kWave;
            const int half = (first ? len1 : n - len1) / 2;
            // position i - 1 lies outside the reversed path (at most n / 2 long)
            const int pl = mi == 0 ? n - 1 : mi - 1;
            int x = 0;
            if (kLen && rt == 0) x = tour[pl];
            for (int q = rt; q < half; q += rthr) {
                int p = mi + q;
                if (p >= n) p -= n;
                int r = mj - q;
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
            if (kLen && rt == 0) {
                // the two new edges close the reversed path: {a, c} and
                // {a1, c1}, the one next to the city left of it first
                const bool left_ac = x == mv.a || x == mv.c;
                elen[pl] = left_ac ? mv.dac : mv.da1c1;
                elen[mj] = left_ac ? mv.da1c1 : mv.dac;
            }
        }
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
    // more waves shorten the reversal of long paths and cost a little more
    // at the barriers: 4 below 1024 cities, 8 below 8192, 16 from there
    const int waves = s.two_opt_waves ? s.two_opt_waves : s.n < 1024 ? 4 : s.n < 8192 ? 8 : 16;
    return hipLaunchKernel(kern, dim3(s.ants), dim3(64 * waves), args, lds, st);
}

}  // namespace mmas
