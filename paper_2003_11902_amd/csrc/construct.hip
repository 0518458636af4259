// Tour construction (the inner loops of Alg. 1): one ant per wave64.
//
// Each step selects the next city by weighted reservoir sampling (Alg. 4):
// every eligible city v draws u and gets the key ln(u) * (1 / w(cur, v)), the
// reciprocal of the weight computed ahead as Sec. 4.2.2 suggests; the wave
// keeps the largest key, the lowest city among equal keys. Eligible are the
// unvisited cities of the current city's candidate list (Sec. 4.3), one per
// lane, with w = choice_info along the list; when all are visited, every
// unvisited city with w = choice_info[cur][v] (dense trails) or
// tau_min^alpha * eta^beta (candidate-only trails).
//
// The visited set lives in LDS, as a bitmask (one bit per city) or as the
// compact tabu of Sec. 4.1 (one 16-bit entry per city plus the length L).
// Tours are gathered in a register (lane k % 64 holds step k) and stored 64
// cities at a time; tour lengths accumulate at those flushes.
#include <atomic>
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// pointers typed with their address space, so that an LDS read and a global
// read of the same element are never folded into one generic (flat) load
template <class T>
using LdsPtr = __attribute__((address_space(3))) T*;
template <class T>
using GlbPtr = __attribute__((address_space(1))) T*;
constexpr size_t kDrawBytes = 4 * kWave * sizeof(float);  // candidate draws of the next steps
constexpr size_t kScratchBytes = 16;                       // per-ant counter of the fallback list

// ---- tabu variants ---------------------------------------------------------

struct BitmaskTabu {
    uint32_t* bits;
    __device__ void attach(uint8_t* lds, int) { bits = reinterpret_cast<uint32_t*>(lds); }
    __device__ void init(uint8_t* lds, int n, int lane) {
        bits = reinterpret_cast<uint32_t*>(lds);
        const int words = (n + 31) >> 5;
        for (int w = lane; w < words; w += kWave) bits[w] = 0u;
    }
    __device__ __forceinline__ bool visited(uint32_t v) const { return (bits[v >> 5] >> (v & 31u)) & 1u; }
    // ~0 if city v is unvisited, else 0 (a bit-field extract and a decrement)
    __device__ __forceinline__ uint32_t live(uint32_t v) const {
        const uint32_t word = bits[__builtin_amdgcn_ubfe(v, 5u, 11u)];
        return __builtin_amdgcn_ubfe(word, v, 1u) - 1u;  // (the offset is taken mod 32)
    }
    __device__ __forceinline__ void mark(uint32_t v, int lane) {
        if (lane == 0) atomicOr(&bits[v >> 5], 1u << (v & 31u));
    }
};

// Compact tabu: entries[i] for i < L lists the unvisited cities; for i >= L,
// entries[i] is the position of city i if it was moved left, or n once city i
// is visited. City u is visited iff entries[u] > u.
struct CompactTabu {
    uint16_t* entries;
    int L;
    int n;
    __device__ void attach(uint8_t* lds, int n_) {
        entries = reinterpret_cast<uint16_t*>(lds);
        n = n_;
        L = n_;
    }
    __device__ void init(uint8_t* lds, int n_, int lane) {
        entries = reinterpret_cast<uint16_t*>(lds);
        n = n_;
        L = n_;
        for (int i = lane; i < n_; i += kWave) entries[i] = (uint16_t)i;
    }
    __device__ __forceinline__ bool visited(uint32_t v) const { return entries[v] > v; }
    __device__ __forceinline__ uint32_t live(uint32_t v) const { return entries[v] > v ? 0u : ~0u; }
    __device__ __forceinline__ const uint16_t* list() const { return entries; }  // the L unvisited cities
    __device__ __forceinline__ void mark(uint32_t u, int lane) {
        // u is wave-uniform: both cells are read at once (the same for every
        // lane, one LDS round trip) into scalar registers; lane 0 writes
        const int iu_v = entries[u];     // position of u in the left part
        const int t_v = entries[L - 1];  // last city of the left part
        const int iu = __builtin_amdgcn_readfirstlane(iu_v);
        const int t = __builtin_amdgcn_readfirstlane(t_v);
        L = L - 1;
        if (lane == 0) {
            if (iu == L) {
                entries[L] = (uint16_t)n;
            } else {
                entries[iu] = (uint16_t)t;
                entries[t] = (uint16_t)iu;
            }
            if ((int)u != iu) entries[u] = (uint16_t)n;
        }
    }
};

// The list tabu of Sec. 4.1 (after Dawson and Stewart, and Uchida et al.):
// unv[0 .. L) lists the unvisited cities, idx[v] is the position of city v
// in unv; marking v swaps it with the last unvisited entry and shortens the
// list (reading C-18: the swap that the worked example of Sec. 4.1 needs), so
// city v is visited iff idx[v] >= L. 4n bytes.
struct ListTabu {
    uint16_t* unv;
    uint16_t* idx;
    int L;
    __device__ void attach(uint8_t* lds, int n_) {
        unv = reinterpret_cast<uint16_t*>(lds);
        idx = unv + n_;
        L = n_;
    }
    __device__ void init(uint8_t* lds, int n_, int lane) {
        attach(lds, n_);
        for (int i = lane; i < n_; i += kWave) {
            unv[i] = (uint16_t)i;
            idx[i] = (uint16_t)i;
        }
    }
    __device__ __forceinline__ bool visited(uint32_t v) const { return (int)idx[v] >= L; }
    __device__ __forceinline__ uint32_t live(uint32_t v) const { return (int)idx[v] >= L ? 0u : ~0u; }
    __device__ __forceinline__ const uint16_t* list() const { return unv; }
    __device__ __forceinline__ void mark(uint32_t u, int lane) {
        // every lane reads the same cells; lane 0 writes
        const int iu = idx[u];
        L = L - 1;
        const int last = unv[L];
        if (lane == 0) {
            unv[iu] = (uint16_t)last;
            idx[last] = (uint16_t)iu;
            unv[L] = (uint16_t)u;
            idx[u] = (uint16_t)L;
        }
    }
};

// ---- fallback weights --------------------------------------------------------

// A fallback key is ln(u) times the reciprocal of the weight (Sec. 4.2.2).
// The factor functors give that reciprocal: read from the dense matrix of
// reciprocals the update writes, or computed from the distance (trails kept
// along the candidate lists only: every other weight is tau_min^alpha *
// eta^beta).
struct DenseFactor {
    const float* row_inv;
    __device__ __forceinline__ float operator()(uint32_t v) const { return row_inv[v]; }
};

struct CandFactor {
    const int32_t* drow;
    float tmin_a;
    int beta;
    __device__ __forceinline__ float operator()(uint32_t v) const {
        return 1.0f / (tmin_a * heur_from_dist(drow[v], beta));
    }
};

// The weights themselves (the roulette wheel sums them).
struct DenseWeight {
    const float* row;
    __device__ __forceinline__ float operator()(uint32_t v) const { return row[v]; }
};

struct CandWeight {
    const int32_t* drow;
    float tmin_a;
    int beta;
    __device__ __forceinline__ float operator()(uint32_t v) const {
        return tmin_a * heur_from_dist(drow[v], beta);
    }
};

template <int kTabu>
struct TabuOf;
template <>
struct TabuOf<MMAS_TABU_BITMASK> {
    using type = BitmaskTabu;
};
template <>
struct TabuOf<MMAS_TABU_COMPACT> {
    using type = CompactTabu;
};
template <>
struct TabuOf<MMAS_TABU_LIST> {
    using type = ListTabu;
};

__device__ __forceinline__ void keep_best(uint32_t code, uint32_t node, uint32_t& bcode, uint32_t& bnode) {
    if (code > bcode || (code == bcode && node < bnode)) {
        bcode = code;
        bnode = node;
    }
}

// Keys of an all-node fallback over `list` (the L unvisited cities, or a
// part of them): city v draws slot cl + v. Each lane takes four list entries
// per round and issues their weight loads before the Philox and logarithm
// work, so the loads overlap it. Folds the best (code, city) of each lane
// into bcode / bnode.
template <class F>
__device__ __forceinline__ void fallback_keys(const uint16_t* list, int L, const F& factor, int cl, uint64_t seed,
                                              uint32_t it, uint32_t ant, uint32_t step, int lane, uint32_t& bcode,
                                              uint32_t& bnode) {
    for (int base = 0; base < L; base += 4 * kWave) {
        uint32_t v[4];
        float f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * kWave + lane;
            v[u] = i < L ? (uint32_t)list[i] : kNone;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = v[u] != kNone ? factor(v[u]) : 1.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (v[u] == kNone) continue;
            const uint32_t slot = (uint32_t)cl + v[u];
            const Words4 blk = draw_block(seed, it, ant, step, slot);
            const float key = log_u01(u01(pick_word(blk, slot & 3u))) * f[u];
            keep_best(ord_key(key), v[u], bcode, bnode);
        }
    }
}

// All-node fallback over a list of the L unvisited cities (the compact tabu's
// left part).
template <class F>
__device__ __forceinline__ uint32_t fallback_list(const uint16_t* list, int L, const F& factor, int cl, uint64_t seed,
                                                  uint32_t it, uint32_t ant, uint32_t step, int lane) {
    uint32_t bcode = 0u, bnode = kNone;
    fallback_keys(list, L, factor, cl, seed, it, ant, step, lane, bcode, bnode);
    return wave_select<4>(bcode, bnode);
}

// Entries of the list a one-wave fallback over a bitmask tabu builds in LDS
// (unless the launch allows more): the unvisited cities are listed and keyed
// in passes of at most this many, so the ant's LDS does not grow with n.
constexpr int kListCap = 512;
__host__ __device__ inline int list_cap(const Shape& s) {
    return s.list_cap > 0 ? s.list_cap : (s.n < kListCap ? s.n : kListCap);
}

// All-node fallback over a bitmask tabu. Each pass takes the next words (one
// per lane, at most 64), keeps the longest run of them whose unvisited cities
// fit in `cap` list entries (a wave prefix sum of their counts gives every
// lane its first slot), lists those cities and keys them; the best key over
// all passes wins (largest key, lowest city), as over one list of them all.
template <class F>
__device__ __forceinline__ uint32_t fallback_bitmask(const BitmaskTabu& tabu, int n, uint16_t* list, int cap,
                                                     const F& factor, int cl, uint64_t seed, uint32_t it, uint32_t ant,
                                                     uint32_t step, int lane) {
    const int words = (n + 31) >> 5;
    uint32_t bcode = 0u, bnode = kNone;
    for (int w0 = 0; w0 < words;) {
        const int wi = w0 + lane;
        uint32_t fr = 0u;
        if (wi < words) {
            fr = ~tabu.bits[wi];
            if (wi == words - 1 && (n & 31)) fr &= (1u << (n & 31)) - 1u;
        }
        const int cnt = __popc(fr);
        const int incl = wave_incl_scan(cnt, lane);
        // a prefix of the lanes (incl grows with the lane); lane 0 always
        // fits, since one word holds at most 32 <= cap cities
        const bool fits = (wi < words) & (incl <= cap);
        const int nfit = __popcll(__ballot(fits));
        const int L = __builtin_amdgcn_readlane(incl, nfit - 1);
        if (fits) {
            int p = incl - cnt;
            while (fr) {
                const int b = __ffs(fr) - 1;
                fr &= fr - 1u;
                list[p++] = (uint16_t)(wi * 32 + b);
            }
        }
        fallback_keys(list, L, factor, cl, seed, it, ant, step, lane, bcode, bnode);
        w0 += nfit;
    }
    return wave_select<4>(bcode, bnode);
}

// A wave's best (key code, lowest city) packed so that the larger value is
// the better one; 0 if the wave saw no city.
__device__ __forceinline__ unsigned long long share_result(uint32_t bcode, uint32_t bnode) {
    const uint32_t bc = wave_max_u32<4>(bcode);
    if (bc == 0u) return 0ull;
    const uint64_t tied = __ballot(bcode == bc);
    uint32_t node;
    if (__popcll(tied) == 1)
        node = (uint32_t)__builtin_amdgcn_readlane((int)bnode, __ffsll((unsigned long long)tied) - 1);
    else
        node = wave_min_u32<4>(bcode == bc ? bnode : kNone);
    return ((unsigned long long)bc << 32) | (unsigned long long)(~node);
}

// The all-node fallback of the single-colony kernel, outlined (it is rare
// with a list, and one copy serves every step of the unrolled step loop):
// the same keys and winner as fallback_bitmask / fallback_list, but with the
// LDS tabu and the global factor row passed with their address spaces (an
// outlined function would otherwise reach both through flat accesses) and
// without branches around a lane's keys. Two layouts:
//  - by list entries: a lane keys four entries of the list of the L
//    unvisited cities a round (the compact and list tabus keep that list,
//    the bitmask tabu's unvisited cities are listed into `list` first), one
//    Philox block per entry;
//  - by draw blocks: a lane takes the block of slots 4b .. 4b+3 a round,
//    computes it once and keys each of its cities that is unvisited (every
//    city is looked at, but a block serves four).
// The cheaper one by instruction count is taken: a round of blocks costs a
// Philox block (about 45) and four keys (about 45 each with the tabu test);
// the list costs a Philox block and a key (about 85) for every 64 entries
// (rounds whose entries are all past L are skipped), plus about 140 to list
// a bitmask. `tabu`: the bitmask words,
// the compact tabu's entries or the list tabu's unv (idx follows at n);
// L: the number of unvisited cities. Key factors: irow[v], the reciprocal of
// the weight (dense trails), or 1 / (tmin_a * eta(drow[v])^beta)
// (candidate-only trails).
// Wave-uniform values that arrive in vector registers (the arguments of an
// outlined function) read back into scalar registers, so that the branches
// and loops over them are scalar.
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ float uni(float x) { return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x))); }
__device__ __forceinline__ uint64_t uni(uint64_t x) {
    return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}
template <class T>
__device__ __forceinline__ T* uni_ptr(T* p) {
    return reinterpret_cast<T*>(uni((uint64_t)reinterpret_cast<uintptr_t>(p)));
}

template <int kTabu, int kPher>
__device__ __attribute__((noinline)) uint32_t fallback_lone(LdsPtr<const uint16_t> tabu_v, LdsPtr<uint16_t> list_v,
                                                            int L_v, int n_v, GlbPtr<const float> irow_v,
                                                            GlbPtr<const int32_t> drow_v, float tmin_a_v, int beta_v,
                                                            int cl_v, uint64_t seed_v, uint32_t it_v, uint32_t ant_v,
                                                            uint32_t step_v, int lane) {
    constexpr bool kList = kTabu != MMAS_TABU_BITMASK;
    const LdsPtr<const uint16_t> tabu = (LdsPtr<const uint16_t>)uni((uint32_t)(uintptr_t)tabu_v);
    const LdsPtr<uint16_t> list = (LdsPtr<uint16_t>)uni((uint32_t)(uintptr_t)list_v);
    const GlbPtr<const float> irow = (GlbPtr<const float>)uni((uint64_t)(uintptr_t)irow_v);
    const GlbPtr<const int32_t> drow = (GlbPtr<const int32_t>)uni((uint64_t)(uintptr_t)drow_v);
    int L = uni(L_v);
    const int n = uni(n_v), beta = uni(beta_v), cl = uni(cl_v);
    const float tmin_a = uni(tmin_a_v);
    const uint64_t seed = uni(seed_v);
    const uint32_t it = uni(it_v), ant = uni(ant_v), step = uni(step_v);
    auto factor = [&](uint32_t v) -> float {
        if constexpr (kPher == MMAS_PHER_DENSE)
            return irow[v];
        else
            return 1.0f / (tmin_a * heur_from_dist(drow[v], beta));
    };
    const int b_lo = cl >> 2, nb = ((cl + n - 1) >> 2) - b_lo + 1;  // blocks holding slots cl .. cl + n - 1
    const int rounds_b = (nb + kWave - 1) / kWave, per_lane = (L + kWave - 1) / kWave;
    uint32_t bcode = 0u, bnode = kNone;
    if (225 * rounds_b < 85 * per_lane + (kList ? 0 : 140)) {
        for (int b0 = b_lo; b0 < b_lo + nb; b0 += kWave) {
            const int b = b0 + lane;
            uint32_t v[4];
            bool ok[4];
            float f[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * b + j - cl;
                ok[j] = b < b_lo + nb && c >= 0 && c < n;
                v[j] = ok[j] ? (uint32_t)c : 0u;
            }
            // the tabu and factor loads go out before the draws
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                bool seen;
                if constexpr (kTabu == MMAS_TABU_BITMASK) {
                    const LdsPtr<const uint32_t> bits = (LdsPtr<const uint32_t>)tabu;
                    seen = (bits[v[j] >> 5] >> (v[j] & 31u)) & 1u;
                } else if constexpr (kTabu == MMAS_TABU_COMPACT) {
                    seen = tabu[v[j]] > v[j];
                } else {
                    seen = (int)tabu[n + v[j]] >= L;
                }
                ok[j] = ok[j] & !seen;
                f[j] = factor(v[j]);
            }
            const Words4 blk = draw_block(seed, it, ant, step, (uint32_t)(4 * b));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float key = log_u01(u01(blk.w[j])) * f[j];
                keep_best(ok[j] ? ord_key(key) : 0u, v[j], bcode, bnode);
            }
        }
        return wave_select<4>(bcode, bnode);
    }
    if constexpr (!kList) {
        // every unvisited city in ascending order (one pass: room for n),
        // lane l taking 16-bit halves l, l + 64, ... of the bitmask, so that
        // a lane writes at most 16 entries
        const LdsPtr<const uint16_t> halves = tabu;
        const int nh = (n + 15) >> 4;
        L = 0;
        for (int h0 = 0; h0 < nh; h0 += kWave) {
            const int hi = h0 + lane;
            uint32_t fr = 0u;
            if (hi < nh) {
                fr = ~(uint32_t)halves[hi] & 0xFFFFu;
                if (hi == nh - 1 && (n & 15)) fr &= (1u << (n & 15)) - 1u;
            }
            const int cnt = __popc(fr);
            const int incl = wave_incl_scan(cnt, lane);
            int p = L + incl - cnt;
            while (fr) {
                const int b = __ffs(fr) - 1;
                fr &= fr - 1u;
                list[p++] = (uint16_t)(hi * 16 + b);
            }
            L += __builtin_amdgcn_readlane(incl, 63);
        }
    }
    for (int base = 0; base < L; base += 4 * kWave) {
        uint32_t v[4];
        float f[4];
        bool ok[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * kWave + lane;
            ok[u] = i < L;
            v[u] = list[ok[u] ? i : 0];
        }
        // the factor loads go out before the draws and their logarithms
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = factor(v[u]);
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t slot = (uint32_t)cl + v[u];
            const Words4 blk = draw_block(seed, it, ant, step, slot);
            const float key = log_u01(u01(pick_word(blk, slot & 3u))) * f[u];
            const uint32_t code = ok[u] ? ord_key(key) : 0u;
            keep_best(code, v[u], bcode, bnode);
        }
    }
    return wave_select<4>(bcode, bnode);
}

// The same fallback for the compact and list tabus, split between `parts`
// waves that call this with part = 0 .. parts - 1 and the same other
// arguments (a single-colony ant's wave and its draw helper): each keys its
// share (alternate rounds of blocks, or alternate 64-entry chunks of the
// tabu's list, a round holding up to four) and the best of the parts'
// results is the winner. Returns this part's best as share_result packs it.
template <int kTabu, int kPher>
__device__ __attribute__((noinline)) unsigned long long fallback_half(
    LdsPtr<const uint16_t> tabu_v, LdsPtr<const uint16_t> list_v, int L_v, int n_v, GlbPtr<const float> irow_v,
    GlbPtr<const int32_t> drow_v, float tmin_a_v, int beta_v, int cl_v, uint64_t seed_v, uint32_t it_v,
    uint32_t ant_v, uint32_t step_v, int part_v, int parts_v, int lane) {
    static_assert(kTabu != MMAS_TABU_BITMASK, "the tabu keeps the list of unvisited cities");
    const LdsPtr<const uint16_t> tabu = (LdsPtr<const uint16_t>)uni((uint32_t)(uintptr_t)tabu_v);
    const LdsPtr<const uint16_t> list = (LdsPtr<const uint16_t>)uni((uint32_t)(uintptr_t)list_v);
    const GlbPtr<const float> irow = (GlbPtr<const float>)uni((uint64_t)(uintptr_t)irow_v);
    const GlbPtr<const int32_t> drow = (GlbPtr<const int32_t>)uni((uint64_t)(uintptr_t)drow_v);
    const int L = uni(L_v);
    const int n = uni(n_v), beta = uni(beta_v), cl = uni(cl_v);
    const float tmin_a = uni(tmin_a_v);
    const uint64_t seed = uni(seed_v);
    const uint32_t it = uni(it_v), ant = uni(ant_v), step = uni(step_v);
    const int part = uni(part_v), parts = uni(parts_v);
    auto factor = [&](uint32_t v) -> float {
        if constexpr (kPher == MMAS_PHER_DENSE)
            return irow[v];
        else
            return 1.0f / (tmin_a * heur_from_dist(drow[v], beta));
    };
    const int b_lo = cl >> 2, nb = ((cl + n - 1) >> 2) - b_lo + 1;  // blocks holding slots cl .. cl + n - 1
    const int span = kWave * parts;
    const int rounds_b = (nb + span - 1) / span, per_lane = (L + span - 1) / span;
    uint32_t bcode = 0u, bnode = kNone;
    if (225 * rounds_b < 85 * per_lane) {
        for (int b0 = b_lo + part * kWave; b0 < b_lo + nb; b0 += span) {
            const int b = b0 + lane;
            uint32_t v[4];
            bool ok[4];
            float f[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = 4 * b + j - cl;
                ok[j] = b < b_lo + nb && c >= 0 && c < n;
                v[j] = ok[j] ? (uint32_t)c : 0u;
            }
            // the tabu and factor loads go out before the draws
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const bool seen = kTabu == MMAS_TABU_COMPACT ? tabu[v[j]] > v[j] : (int)tabu[n + v[j]] >= L;
                ok[j] = ok[j] & !seen;
                f[j] = factor(v[j]);
            }
            const Words4 blk = draw_block(seed, it, ant, step, (uint32_t)(4 * b));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const float key = log_u01(u01(blk.w[j])) * f[j];
                keep_best(ok[j] ? ord_key(key) : 0u, v[j], bcode, bnode);
            }
        }
        return share_result(bcode, bnode);
    }
    // By list entries (the tabu's list of the L unvisited cities), in chunks
    // of 64: this part takes chunks part, part + parts, ...
    const int c0 = part, cs = parts;
    // U chunks a round (U <= 4): the factor loads go out before the draws
    // and their logarithms
    auto key_round = [&](auto u_tag, int c) {
        constexpr int U = decltype(u_tag)::value;
        uint32_t v[U];
        float f[U];
        bool ok[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = (c + u * cs) * kWave + lane;
            ok[u] = i < L;
            v[u] = list[ok[u] ? i : 0];
        }
#pragma unroll
        for (int u = 0; u < U; ++u) f[u] = factor(v[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t slot = (uint32_t)cl + v[u];
            const Words4 blk = draw_block(seed, it, ant, step, slot);
            const float key = log_u01(u01(pick_word(blk, slot & 3u))) * f[u];
            const uint32_t code = ok[u] ? ord_key(key) : 0u;
            keep_best(code, v[u], bcode, bnode);
        }
    };
    const int chunks = (L + kWave - 1) / kWave;
    int left = chunks > c0 ? (chunks - c0 + cs - 1) / cs : 0;  // this part's chunks
    int c = c0;
    for (; left >= 4; left -= 4, c += 4 * cs) key_round(std::integral_constant<int, 4>{}, c);
    if (left == 3)
        key_round(std::integral_constant<int, 3>{}, c);
    else if (left == 2)
        key_round(std::integral_constant<int, 2>{}, c);
    else if (left == 1)
        key_round(std::integral_constant<int, 1>{}, c);
    return share_result(bcode, bnode);
}

// ---- several waves per ant: the fallback shared by the workgroup ----------

// What the leading wave (the one taking the steps) hands to the helper waves
// of its workgroup for a fallback, and their per-wave results.
struct __align__(16) WideStep {
    int k;               // the step that needs the fallback
    uint32_t cur;        // current city
    int L;               // compact and list tabus: unvisited count
    int stop;            // the tour is done: every wave leaves
};
struct WideLds {
    WideStep step;       // written by the leading wave before the first barrier
                         // of a fallback, read by all after it
    uint32_t counter;    // bitmask tabu: list fill counter
    unsigned long long res[16];  // per wave: (key code << 32) | ~city, 0 = none
};

// The unvisited cities of a bitmask tabu gathered by the whole workgroup
// (thread t takes words t, t + threads, ...): a wave places its words' cities
// by a prefix sum of their counts and claims room for all of them with one
// LDS atomic; `counter` is 0 on entry.
__device__ void gather_unvisited_block(const BitmaskTabu& tabu, int n, uint16_t* list, uint32_t* counter) {
    const int words = (n + 31) >> 5;
    const int lane = (int)(threadIdx.x & 63);
    for (int w0 = (int)(threadIdx.x & ~63u); w0 < words; w0 += (int)blockDim.x) {
        const int wi = w0 + lane;
        uint32_t fr = 0u;
        if (wi < words) {
            fr = ~tabu.bits[wi];
            if (wi == words - 1 && (n & 31)) fr &= (1u << (n & 31)) - 1u;
        }
        const int cnt = __popc(fr);
        const int incl = wave_incl_scan(cnt, lane);
        const int tot = __builtin_amdgcn_readlane(incl, 63);
        if (tot == 0) continue;
        uint32_t base = 0u;
        if (lane == 0) base = atomicAdd(counter, (uint32_t)tot);
        int p = __builtin_amdgcn_readfirstlane((int)base) + incl - cnt;
        while (fr) {
            const int b = __ffs(fr) - 1;
            fr &= fr - 1u;
            list[p++] = (uint16_t)(wi * 32 + b);
        }
    }
}


// This wave's share of a workgroup-wide fallback (entries wave*64 + lane,
// then every 64*waves): its best (key code, lowest city), packed so that the
// larger value is the better one; 0 if the wave saw no city.
template <class F>
__device__ __forceinline__ unsigned long long fallback_share(const uint16_t* list, int L, const F& factor, int cl, uint64_t seed,
                                             uint32_t it, uint32_t ant, uint32_t step, int lane, int wv, int nw) {
    uint32_t bcode = 0u, bnode = kNone;
    const int stride = kWave * nw;
    for (int base = wv * kWave; base < L; base += 4 * stride) {
        uint32_t v[4];
        float f[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int i = base + u * stride + lane;
            v[u] = i < L ? (uint32_t)list[i] : kNone;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) f[u] = v[u] != kNone ? factor(v[u]) : 1.0f;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (v[u] == kNone) continue;
            const uint32_t slot = (uint32_t)cl + v[u];
            const Words4 blk = draw_block(seed, it, ant, step, slot);
            const float key = log_u01(u01(pick_word(blk, slot & 3u))) * f[u];
            keep_best(ord_key(key), v[u], bcode, bnode);
        }
    }
    return share_result(bcode, bnode);
}

// The same share laid out by draw blocks instead of list entries: a lane
// takes the block of slots 4b .. 4b+3 (b from the first block holding slot
// cl, wave*64 + lane, then every 64*waves), computes that Philox block once
// and keys each of its cities (slot - cl) that is unvisited. While most
// cities are unvisited this needs a quarter of the blocks of the list layout;
// the keys, and so the winner, are the same.
template <class T, class F>
__device__ __forceinline__ unsigned long long fallback_share_blocks(const T& tabu, int n, const F& factor, int cl,
                                                                    uint64_t seed, uint32_t it, uint32_t ant,
                                                                    uint32_t step, int lane, int wv, int nw) {
    uint32_t bcode = 0u, bnode = kNone;
    const int b_lo = cl >> 2, b_hi = (cl + n - 1) >> 2;  // blocks holding slots cl .. cl + n - 1
    for (int b0 = b_lo + wv * kWave; b0 <= b_hi; b0 += kWave * nw) {
        const int b = b0 + lane;
        if (b <= b_hi) {
            const Words4 blk = draw_block(seed, it, ant, step, (uint32_t)(4 * b));
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int v = 4 * b + j - cl;
                if (v < 0 || v >= n || tabu.visited((uint32_t)v)) continue;
                const float key = log_u01(u01(blk.w[j])) * factor((uint32_t)v);
                keep_best(ord_key(key), (uint32_t)v, bcode, bnode);
            }
        }
    }
    return share_result(bcode, bnode);
}

// LDS layout of one workgroup: the candidate table of cities 0..R-1 (ids,
// then choice_info), then one region per ant (its draws, its tabu and, for
// the bitmask, room to list the unvisited cities during a fallback).
struct Lds {
    int rows;          // R: rows of the candidate table held in LDS
    int table_bytes;   // bytes of the table part (16-aligned)
    int per_ant;       // bytes of one ant's region
};

__host__ __device__ inline int align16(int x) { return (x + 15) & ~15; }

// The whole workgroup copies the first R rows of the candidate table (ids,
// then the reciprocals of choice_info) into LDS; the caller synchronises.
__device__ void stage_table(const Views& vw, int cl, int R, uint16_t* tcand, float* tchc) {
    const int ne = R * cl;
    for (int e = threadIdx.x; e < ne; e += blockDim.x) {
        tcand[e] = vw.cand[e];
        tchc[e] = vw.chc_inv[e];
    }
}

// One wave's share of a workgroup-wide fallback at step k from city fcur
// (the bitmask tabu's unvisited cities are first gathered by the whole
// workgroup, with a barrier): the wave's best (key code, ~city), 0 if none.
template <int kTabu, int kPher, class T>
__device__ unsigned long long wide_share(const Views& vw, const Shape& s, uint32_t it, int ant, int k, uint32_t fcur,
                                         int L, T& tabu, uint16_t* ulist, WideLds* wl, float tmin_a, int lane, int wv,
                                         int nw) {
    const int n = s.n, cl = s.cl;
    const uint16_t* list;
    if constexpr (kTabu == MMAS_TABU_BITMASK) {
        gather_unvisited_block(tabu, n, ulist, &wl->counter);
        __syncthreads();
        L = __builtin_amdgcn_readfirstlane((int)wl->counter);
        list = ulist;
    } else {
        list = tabu.list();
        if constexpr (kTabu == MMAS_TABU_LIST) tabu.L = L;  // the helpers' copy of the length
    }
    // by draw blocks while they are cheaper: a block costs about a Philox
    // and four keys, a listed city a Philox and one key
    const bool by_blocks = kTabu != MMAS_TABU_BITMASK && 46 * L > 25 * n;
    if constexpr (kPher == MMAS_PHER_DENSE) {
        const DenseFactor wt{vw.choice_inv + (size_t)fcur * n};
        return by_blocks ? fallback_share_blocks(tabu, n, wt, cl, s.seed, it, (uint32_t)ant, (uint32_t)k, lane, wv, nw)
                         : fallback_share(list, L, wt, cl, s.seed, it, (uint32_t)ant, (uint32_t)k, lane, wv, nw);
    } else {
        const CandFactor wt{vw.dist + (size_t)fcur * n, tmin_a, s.beta};
        return by_blocks ? fallback_share_blocks(tabu, n, wt, cl, s.seed, it, (uint32_t)ant, (uint32_t)k, lane, wv, nw)
                         : fallback_share(list, L, wt, cl, s.seed, it, (uint32_t)ant, (uint32_t)k, lane, wv, nw);
    }
}

// The helper waves of a workgroup-wide ant: they wait at the barrier until
// the leading wave posts a fallback (or the end of its tour), key their share
// and post their best, so the steps without a fallback need no barrier.
template <int kTabu, int kPher>
__device__ void wide_helpers(const Views& vw, const Shape& s, uint32_t it, int ant, int lane, uint8_t* region,
                             WideLds* wl, int wv, int nw) {
    const int n = s.n;
    typename TabuOf<kTabu>::type tabu;
    tabu.attach(region + kDrawBytes + kScratchBytes, n);
    uint16_t* ulist = reinterpret_cast<uint16_t*>(region + kDrawBytes + kScratchBytes + align16(4 * ((n + 31) / 32)));
    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    for (;;) {
        __syncthreads();  // a posted fallback, or the end
        const WideStep st = wl->step;
        if (__builtin_amdgcn_readfirstlane(st.stop)) return;
        const unsigned long long mine =
            wide_share<kTabu, kPher>(vw, s, it, ant, __builtin_amdgcn_readfirstlane(st.k),
                                     (uint32_t)__builtin_amdgcn_readfirstlane((int)st.cur),
                                     __builtin_amdgcn_readfirstlane(st.L), tabu, ulist, wl, tmin_a, lane, wv, nw);
        if (lane == 0) wl->res[wv] = mine;
        __syncthreads();  // the results (read by the leading wave)
    }
}

// The leading wave's side of a workgroup-wide fallback at step k from city
// cur: posts it, keys its share with the helpers, and takes the best over
// the waves (the largest key code, then the lowest city); kNone if none.
template <int kTabu, int kPher, class T>
__device__ uint32_t wide_lead_fallback(const Views& vw, const Shape& s, uint32_t it, int ant, int k, uint32_t cur,
                                       T& tabu, uint16_t* ulist, WideLds* wl, float tmin_a, int lane, int nw) {
    if (lane == 0) {
        WideStep st;
        st.k = k;
        st.cur = cur;
        st.L = 0;
        if constexpr (kTabu != MMAS_TABU_BITMASK) st.L = tabu.L;
        st.stop = 0;
        wl->step = st;
        if constexpr (kTabu == MMAS_TABU_BITMASK) wl->counter = 0u;
    }
    __syncthreads();
    int L = 0;
    if constexpr (kTabu != MMAS_TABU_BITMASK) L = tabu.L;
    const unsigned long long mine = wide_share<kTabu, kPher>(vw, s, it, ant, k, cur, L, tabu, ulist, wl, tmin_a, lane, 0, nw);
    if (lane == 0) wl->res[0] = mine;
    __syncthreads();
    // (the record, the counter and the list are read before the second
    // barrier; res is written again only after the next fallback's first)
    const unsigned long long r = lane < nw ? wl->res[lane] : 0ull;
    const uint32_t hi = (uint32_t)(r >> 32), lo = (uint32_t)r;
    const uint32_t mx = wave_max_u32<2>(hi);
    uint32_t best_lo;
    const uint64_t tied = __ballot(hi == mx && lane < nw);
    if (__popcll(tied) == 1)
        best_lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, __ffsll((unsigned long long)tied) - 1);
    else
        best_lo = wave_max_u32<2>(hi == mx ? lo : 0u);
    return mx ? ~best_lo : kNone;
}

// The end of the leading wave's tour: the helpers leave.
__device__ void wide_lead_end(WideLds* wl, int lane) {
    if (lane == 0) {
        WideStep st;
        st.k = 0;
        st.cur = 0u;
        st.L = 0;
        st.stop = 1;
        wl->step = st;
    }
    __syncthreads();
}

// ---- the draw helper of a single-colony ant --------------------------------
//
// A second wave per ant computes the draws (Philox blocks and logarithms) of
// each group of S = 64 / G steps into one of two LDS buffers, a group ahead
// of the ant's wave, which then only reads them; with the compact tabu
// (kHelpShare) it also keys half of every all-city fallback (fallback_half's
// part 1) while the ant's wave keys the other half. Counters in LDS hand the
// buffers and the fallbacks over: the helper writes group g once group
// g - 2 is read, and serves a posted fallback whenever it waits. Waits are
// bounded: past the limit the ant's wave flags the tour (state flag 32) and
// keys the rest alone, and the helper leaves, so no wave can wait for ever.
// Both waves must read any counter the other writes through lds_get (a
// volatile LDS read) and write their own through lds_put.
struct HelpLds {
    int made;                // draw groups written (helper)
    int read;                // draw groups read (ant's wave)
    int req;                 // fallbacks posted (ant's wave)
    int done;                // fallbacks whose part 1 is keyed (helper)
    int k;                   // the posted fallback: step,
    uint32_t cur;            // current city,
    int L;                   // unvisited cities,
    int stop;                // and 1 once the tour is done (the helper leaves)
    unsigned long long res;  // part 1's best (share_result) of fallback `done`
    int pad[2];              // (to 48 bytes)
};
static_assert(sizeof(HelpLds) == 48, "16-byte multiple");
constexpr size_t kHelpBytes = kDrawBytes + sizeof(HelpLds);  // second draw buffer, then the counters
constexpr int kHelpSpins = 1 << 24;                          // sleeps of 64 clocks before a wait gives up
// The tabus whose fallbacks the helper shares: measured at n = 1002, the
// shared fallback made the compact tabu's construction about 7 % faster; the
// bitmask tabu's it made 1-3 % slower and the list tabu's no faster.
template <int kTabu>
constexpr bool kHelpShare = kTabu == MMAS_TABU_COMPACT;

__device__ __forceinline__ int lds_get(const int* c) {
    return __builtin_amdgcn_readfirstlane(*(LdsPtr<volatile const int>)c);
}
__device__ __forceinline__ void lds_put(int* c, int v) {
    asm volatile("" ::: "memory");
    *(LdsPtr<volatile int>)c = v;
}

// waits until the LDS counter c reaches `want`; false if it gave up
__device__ __forceinline__ bool wait_count(const int* c, int want) {
    for (int spins = 0; spins < kHelpSpins; ++spins) {
        if (lds_get(c) >= want) {
            asm volatile("" ::: "memory");
            return true;
        }
        __builtin_amdgcn_s_sleep(1);
    }
    return false;
}

// Part `part` of two of the all-city fallback of step k from city cur with
// L unvisited cities, on the list of the ant's tabu (compact or list).
template <int kTabu, int kPher, class T>
__device__ __forceinline__ unsigned long long half_part(const Views& vw, const Shape& s, uint32_t it, int ant, int k,
                                                        uint32_t cur, int L, const T& tabu, float tmin_a, int part,
                                                        int lane) {
    const int n = s.n;
    // (C-style casts: the only casts that change the address space)
    const GlbPtr<const float> irow =
        kPher == MMAS_PHER_DENSE ? (GlbPtr<const float>)(vw.choice_inv + (size_t)cur * n) : nullptr;
    const GlbPtr<const int32_t> drow =
        kPher == MMAS_PHER_DENSE ? nullptr : (GlbPtr<const int32_t>)(vw.dist + (size_t)cur * n);
    const LdsPtr<const uint16_t> lv = (LdsPtr<const uint16_t>)tabu.list();
    return fallback_half<kTabu, kPher>(lv, lv, L, n, irow, drow, tmin_a, s.beta, s.cl, s.seed, it, (uint32_t)ant,
                                       (uint32_t)k, part, 2, lane);
}

// The helper wave of ant `ant`: `region` is the ant's region (draw buffer 0
// at its start, the tabu after it), `help` the helper's part (draw buffer 1,
// then the HelpLds).
template <int kTabu, int kPher, int kG>
__device__ void draw_helper(const Views& vw, const Shape& s, uint32_t it, int ant, int lane, uint8_t* region,
                            uint8_t* help) {
    constexpr int gsh = kG == 1 ? 0 : kG == 2 ? 1 : kG == 4 ? 2 : kG == 8 ? 3 : 4;
    constexpr int S = kWave >> gsh;
    const int n = s.n;
    float* buf0 = reinterpret_cast<float*>(region);
    float* buf1 = reinterpret_cast<float*>(help);
    HelpLds* h = reinterpret_cast<HelpLds*>(help + kDrawBytes);
    typename TabuOf<kTabu>::type tabu;
    tabu.attach(region + kDrawBytes + kScratchBytes, n);
    float tmin_a = 0.0f;
    if (kHelpShare<kTabu> && kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    int served = 0;
    // keys part 1 of a posted fallback, if there is one; true if it did
    auto serve = [&]() -> bool {
        if constexpr (!kHelpShare<kTabu>) {
            return false;
        } else {
            const int r = lds_get(&h->req);
            if (r <= served) return false;
            asm volatile("" ::: "memory");
            const unsigned long long res =
                half_part<kTabu, kPher>(vw, s, it, ant, lds_get(&h->k), (uint32_t)lds_get(reinterpret_cast<int*>(&h->cur)),
                                        lds_get(&h->L), tabu, tmin_a, 1, lane);
            asm volatile("" ::: "memory");
            *(LdsPtr<volatile unsigned long long>)&h->res = res;
            asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the result is in LDS before the count
            lds_put(&h->done, r);
            served = r;
            return true;
        }
    };
    // waits until the counter c reaches `want`, serving fallbacks meanwhile;
    // false if it gave up
    auto wait_serving = [&](const int* c, int want) -> bool {
        for (int spins = 0; spins < kHelpSpins; ++spins) {
            if (serve()) spins = 0;
            if (lds_get(c) >= want) {
                asm volatile("" ::: "memory");
                return true;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        return false;
    };
    const int groups = (n + S - 1) / S;
    for (int g = 0; g < groups; ++g) {
        const Words4 b = draw_block(s.seed, it, (uint32_t)ant, (uint32_t)(g * S + (lane >> gsh)),
                                    (uint32_t)(4 * (lane & (kG - 1))));
        float4 lv;
        lv.x = log_u01(u01(b.w[0]));
        lv.y = log_u01(u01(b.w[1]));
        lv.z = log_u01(u01(b.w[2]));
        lv.w = log_u01(u01(b.w[3]));
        // (computed before the wait, so that the waits serve fallbacks at once)
        asm volatile("" : "+v"(lv.x), "+v"(lv.y), "+v"(lv.z), "+v"(lv.w));
        // the buffer of group g held group g - 2
        if (g >= 2 && !wait_serving(&h->read, g - 1)) return;
        *reinterpret_cast<float4*>(((g & 1) ? buf1 : buf0) + 4 * lane) = lv;
        asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the draws are in LDS before the count
        lds_put(&h->made, g + 1);
    }
    // every group is written: serve fallbacks until the tour is done
    wait_serving(&h->stop, 1);
}

// One ant's tour (one wave64, the batched kernel's step): start city, n - 1
// selection steps, tour and length stores. `region` is the ant's LDS region;
// rows 0..R-1 of the candidate table are in LDS at tcand / tchc.
template <int kTabu, int kPher>
__device__ void construct_ant(const Views& vw, const Shape& s, uint32_t it, int ant, int lane, uint8_t* region,
                              const uint16_t* tcand, const float* tchc, int R) {
    const int n = s.n, cl = s.cl;
    const uint64_t seed = s.seed;

    // per-ant LDS: the draws of the next steps (256 floats), then the tabu
    float* lnbuf = reinterpret_cast<float*>(region);
    typename TabuOf<kTabu>::type tabu;
    tabu.init(region + kDrawBytes + kScratchBytes, n, lane);
    uint16_t* ulist = reinterpret_cast<uint16_t*>(region + kDrawBytes + kScratchBytes + align16(4 * ((n + 31) / 32)));

    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    // (C-style casts: the only casts that change the address space)
    const LdsPtr<const uint16_t> lds_cand = (LdsPtr<const uint16_t>)tcand;
    const LdsPtr<const float> lds_chc = (LdsPtr<const float>)tchc;
    const GlbPtr<const uint16_t> glb_cand = (GlbPtr<const uint16_t>)vw.cand;
    const GlbPtr<const float> glb_chc = (GlbPtr<const float>)vw.chc_inv;  // reciprocals

    // start city: floor(x * n / 2^32) of draw (step 0, slot 0)
    const uint32_t x0 = draw_block(seed, it, (uint32_t)ant, 0u, 0u).w[0];
    const uint32_t start = (uint32_t)(((uint64_t)x0 * (uint64_t)n) >> 32);
    tabu.mark(start, lane);

    // Candidate draws are generated ahead, S steps at a time: lane l computes
    // the Philox block of step k + l/G and slots 4(l%G)..4(l%G)+3 and stores
    // their logarithms at lnbuf[4l..4l+3]; step k + j then reads slot r at
    // lnbuf[4jG + r]. G = 4-slot groups per step (a power of two), S = 64/G.
    const int gsh = cl <= 4 ? 0 : cl <= 8 ? 1 : cl <= 16 ? 2 : cl <= 32 ? 3 : 4;
    const int G = 1 << gsh;
    const int S = kWave >> gsh;

    uint16_t* tour_out = vw.tours + (size_t)ant * n;
    const int32_t* dist = vw.dist;
    uint32_t tbuf = start;   // lane (k & 63) holds the city of step k
    uint32_t prev_last = 0;  // last city of the previous 64-step chunk
    int64_t len = 0;
    int64_t fb_steps = 0, fb_nodes = 0;
    uint32_t cur = start;

    for (int k = 1; k < n; ++k) {
        uint32_t next = kNone;
        if (cl > 0) {
            // candidate phase: lane r holds rank r of cur's list
            // every lane loads a valid entry (lanes past the list repeat the
            // last one and get no key); the row comes from LDS or from global
            // memory through separate, address-space-typed loads
            uint32_t node;
            float w;
            const int cs = __builtin_amdgcn_readfirstlane((int)cur);
            const int e = cs * cl + (lane < cl ? lane : cl - 1);
            if (cs < R) {
                node = lds_cand[e];
                w = lds_chc[e];
            } else {
                node = glb_cand[e];
                w = glb_chc[e];
            }
            const int j = (k - 1) & (S - 1);
            if (j == 0) {
                // (steps past n - 1 draw values nobody reads; no lane is masked)
                const int ks = k + (lane >> gsh);
                const Words4 b = draw_block(seed, it, (uint32_t)ant, (uint32_t)ks, (uint32_t)(4 * (lane & (G - 1))));
                float4 lv;
                lv.x = log_u01(u01(b.w[0]));
                lv.y = log_u01(u01(b.w[1]));
                lv.z = log_u01(u01(b.w[2]));
                lv.w = log_u01(u01(b.w[3]));
                *reinterpret_cast<float4*>(lnbuf + 4 * lane) = lv;
            }
            // branch-free: every lane of the list computes its key; visited
            // cities and lanes past the list contribute no key
            const float lnu = lnbuf[4 * j * G + (lane & (4 * G - 1))];
            // the visited-bit load is issued first, then every lane divides (no
            // exec mask), so that the division overlaps the load
            const bool seen = tabu.visited(node);
            float key = lnu * w;  // (w holds 1 / choice_info)
            asm volatile("" : "+v"(key));
            const bool live = (lane < cl) & !seen;  // no short circuit: no exec mask
            const uint32_t code = live ? ord_key(key) : 0u;
            // (all four rows even for cl <= 32: lanes past the list hold no key,
            // and one code path is faster than two)
            next = wave_select_step<4>(code, node);
        }
        if (next == kNone) {
            fb_steps += 1;
            fb_nodes += n - k;
            const int cap = list_cap(s);
            if constexpr (kPher == MMAS_PHER_DENSE) {
                const DenseFactor wt{vw.choice_inv + (size_t)cur * n};
                if constexpr (kTabu == MMAS_TABU_BITMASK)
                    next = fallback_bitmask(tabu, n, ulist, cap, wt, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
                else
                    next = fallback_list(tabu.list(), tabu.L, wt, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
            } else {
                const CandFactor wt{dist + (size_t)cur * n, tmin_a, s.beta};
                if constexpr (kTabu == MMAS_TABU_BITMASK)
                    next = fallback_bitmask(tabu, n, ulist, cap, wt, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
                else
                    next = fallback_list(tabu.list(), tabu.L, wt, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
            }
        }
        if (next >= (uint32_t)n) {
            // unreachable with a validated instance (some unvisited city always
            // has a key); report it instead of indexing out of bounds
            if (lane == 0) atomicOr(&vw.state->flags, 8u);
            break;
        }
        tabu.mark(next, lane);
        const int slot = k & 63;
        if (lane == slot) tbuf = next;
        cur = next;
        if (slot == 63 || k == n - 1) {
            // flush the chunk of steps k0 .. k; lane l holds step k0 + l
            const int k0 = k - slot;
            const uint32_t prev = __shfl_up(tbuf, 1);
            if (lane <= slot) {
                tour_out[k0 + lane] = (uint16_t)tbuf;
                // edge entering step k0 + l (none for step 0)
                const uint32_t from = lane == 0 ? prev_last : prev;
                if (k0 + lane > 0) len += dist[(size_t)from * n + tbuf];
            }
            prev_last = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, slot);
        }
    }
    if (lane == 0) len += dist[(size_t)cur * n + start];  // closing edge
    len = wave_sum_i64(len);
    if (lane == 0) {
        vw.lengths[ant] = len;
        vw.fallback[ant] = fb_steps;
        vw.fallback[s.ants + ant] = fb_nodes;
    }
}

// One ant per wave64 for the single colony, where every wave sits alone on
// its SIMD and the time per step is the length of the step's instruction
// chain. The same selection as construct_ant, laid out so that the chain
// stays short: the current and the next city are wave-uniform (scalar
// registers and scalar branches, no exec-mask bookkeeping around the step);
// the steps run in groups of S (one draw generation per group, no per-step
// test for it) inside chunks of 64 (one tour flush per chunk); the visited
// test folds into the key code as a mask; and for cl <= 32 (kRows = 2) the
// argmax reduces only the two rows that hold the list.
// kWide: the wave leads a workgroup whose other waves share its fallbacks
// (wide_helpers), nw waves in all. kHelp (kG > 0): a draw helper wave
// (draw_helper) fills the draw buffers and keys half of every fallback;
// `help` is its part of the region (second buffer, counters).
template <int kTabu, int kPher, int kRows, int kG, bool kWide = false, bool kHelp = false>
__device__ void construct_lone(const Views& vw, const Shape& s, uint32_t it, int ant, int lane, uint8_t* region,
                               const uint16_t* tcand, const float* tchc, int R, WideLds* wl = nullptr,
                               int nw = 1, uint8_t* help = nullptr) {
    const int n = s.n, cl = s.cl;
    const uint64_t seed = s.seed;
    float* lnbuf = reinterpret_cast<float*>(region);
    typename TabuOf<kTabu>::type tabu;
    tabu.init(region + kDrawBytes + kScratchBytes, n, lane);
    uint16_t* ulist = reinterpret_cast<uint16_t*>(region + kDrawBytes + kScratchBytes + align16(4 * ((n + 31) / 32)));

    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    const LdsPtr<const uint16_t> lds_cand = (LdsPtr<const uint16_t>)tcand;
    const LdsPtr<const float> lds_chc = (LdsPtr<const float>)tchc;
    const GlbPtr<const uint16_t> glb_cand = (GlbPtr<const uint16_t>)vw.cand;
    const GlbPtr<const float> glb_chc = (GlbPtr<const float>)vw.chc_inv;  // reciprocals
    LdsPtr<const float> lds_ln = (LdsPtr<const float>)lnbuf;

    const uint32_t x0 = draw_block(seed, it, (uint32_t)ant, 0u, 0u).w[0];
    const int start = __builtin_amdgcn_readfirstlane((int)(((uint64_t)x0 * (uint64_t)n) >> 32));
    tabu.mark((uint32_t)start, lane);

    // Draws ahead: G 4-slot groups per step, S = 64 / G steps per generation.
    // The generation for the group of steps k0 .. k0 + S - 1 (k0 a multiple
    // of S; step 0 is the start and reads none) has lane l compute the Philox
    // block of step k0 + l / G, slots 4(l % G) .. 4(l % G) + 3, and store
    // their logarithms at lnbuf[4l .. 4l + 3]; step k0 + j reads slot r at
    // lnbuf[4jG + r].
    // (kG > 0: G fixed at compile time, with the draws pipelined below)
    const int gsh = kG == 1 ? 0 : kG == 2 ? 1 : kG == 4 ? 2 : kG == 8 ? 3 : kG == 16 ? 4
                  : cl <= 4 ? 0 : cl <= 8 ? 1 : cl <= 16 ? 2 : cl <= 32 ? 3 : 4;
    const int G = 1 << gsh;
    const int S = kWave >> gsh;
    const int lr = lane < cl ? lane : cl - 1;       // lanes past the list repeat the last entry
    const uint32_t lane_ok = lane < cl ? ~0u : 0u;  // ... and never hold a key
    const int ln_lane = lane & (4 * G - 1);
    // bitmask marks: LDS byte address of each lane's OR (see below)
    uint32_t mark_mask = lane == 0 ? ~0u : 0u;
    uint32_t mark_base = (uint32_t)(uintptr_t)(LdsPtr<uint8_t>)region +
                         (lane == 0 ? (uint32_t)(kDrawBytes + kScratchBytes) : 4u * (uint32_t)lane);
    // (opaque to the compiler, which would otherwise turn the arithmetic
    // below back into lane-0 selects)
    asm volatile("" : "+v"(mark_mask), "+v"(mark_base));

    uint16_t* tour_out = vw.tours + (size_t)ant * n;
    const int32_t* dist = vw.dist;
    uint32_t tbuf = (uint32_t)start;  // lane (k & 63) holds the city of step k
    uint32_t prev_last = 0;           // city of the last step of the previous chunk
    int64_t len = 0;
    int64_t fb_steps = 0, fb_nodes = 0;
    int cur = start;
    bool bad = false;
    bool bad_help = false;  // a wait for the draw helper gave up
    int fseq = 0;           // fallbacks posted to the helper
    HelpLds* hl = kHelp ? reinterpret_cast<HelpLds*>(help + kDrawBytes) : nullptr;

    // the all-city fallback of step k from city cur (rare with a list)
    auto fallback = [&](int k) -> uint32_t {
        // (k laundered so that n - k is not kept as a 64-bit induction
        // variable on every step)
        int kk = k;
        if constexpr (kWide)
            kk = __builtin_amdgcn_readfirstlane(kk);
        else
            asm volatile("" : "+s"(kk));
        fb_steps += 1;
        fb_nodes += n - kk;
        uint32_t pick;
        if constexpr (kWide) {
            pick = wide_lead_fallback<kTabu, kPher>(vw, s, it, ant, kk, (uint32_t)cur, tabu, ulist, wl, tmin_a, lane, nw);
        } else {
            int L = n - kk;
            if constexpr (kTabu != MMAS_TABU_BITMASK) L = tabu.L;
            if constexpr (kHelp && kHelpShare<kTabu>) {
                // post the fallback, key part 0 and take the better of the parts
                ++fseq;
                *reinterpret_cast<int4*>(&hl->k) = make_int4(kk, cur, L, 0);
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the record is in LDS before the count
                lds_put(&hl->req, fseq);
                const unsigned long long r0 =
                    half_part<kTabu, kPher>(vw, s, it, ant, kk, (uint32_t)cur, L, tabu, tmin_a, 0, lane);
                unsigned long long r1;
                if (!bad_help && wait_count(&hl->done, fseq)) {
                    r1 = *(LdsPtr<volatile unsigned long long>)&hl->res;
                } else {  // (never expected) part 1 here too
                    bad_help = true;
                    r1 = half_part<kTabu, kPher>(vw, s, it, ant, kk, (uint32_t)cur, L, tabu, tmin_a, 1, lane);
                }
                const unsigned long long r = r0 > r1 ? r0 : r1;
                pick = r ? ~(uint32_t)r : kNone;
            } else {
                // (C-style casts: the only casts that change the address space)
                const GlbPtr<const float> irow =
                    kPher == MMAS_PHER_DENSE ? (GlbPtr<const float>)(vw.choice_inv + (size_t)cur * n) : nullptr;
                const GlbPtr<const int32_t> drow =
                    kPher == MMAS_PHER_DENSE ? nullptr : (GlbPtr<const int32_t>)(dist + (size_t)cur * n);
                if constexpr (kTabu == MMAS_TABU_BITMASK)
                    pick = fallback_lone<kTabu, kPher>((LdsPtr<const uint16_t>)tabu.bits, (LdsPtr<uint16_t>)ulist, L,
                                                       n, irow, drow, tmin_a, s.beta, cl, seed, it, (uint32_t)ant,
                                                       (uint32_t)k, lane);
                else
                    pick = fallback_lone<kTabu, kPher>((LdsPtr<const uint16_t>)tabu.list(),
                                                       (LdsPtr<uint16_t>)tabu.list(), L, n, irow, drow, tmin_a,
                                                       s.beta, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
            }
        }
        const uint32_t next = (uint32_t)__builtin_amdgcn_readfirstlane((int)pick);
        // no city is unreachable with a validated instance; were it not,
        // report it after the tour and go on with city 0 (the tour is void)
        // rather than index out of bounds
        bad |= next >= (uint32_t)n;
        return next < (uint32_t)n ? next : 0u;
    };

    // marks the chosen city, records it as step k and moves there
    auto advance = [&](uint32_t next, int k) {
        if constexpr (kTabu == MMAS_TABU_BITMASK) {
            // every lane issues the OR, so that no exec mask is set up around
            // it: lane 0 into the city's word, the others a 0 into their own
            // word of the draw buffer (no change)
            const uint32_t addr = mark_base + (((next >> 5) << 2) & mark_mask);
            __hip_atomic_fetch_or((LdsPtr<uint32_t>)(uintptr_t)addr, (1u << (next & 31u)) & mark_mask,
                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        } else {
            tabu.mark(next, lane);
        }
        if (lane == (k & 63)) tbuf = next;
        cur = __builtin_amdgcn_readfirstlane((int)next);
    };

    // The row entry of this lane for city c (rank lr of its candidate list),
    // loaded one step ahead: as soon as the next city is known, before it is
    // marked, so the loads are not queued behind the mark.
    uint16_t node_next = 0;  // (16 bits: widened where it is used, not where the loads meet)
    float w_next = 0.0f;
    auto load_row = [&](int c) {
        const int e = c * cl + lr;
        if (__builtin_expect(c < R, 1)) {
            node_next = lds_cand[e];
            w_next = lds_chc[e];
        } else {
            node_next = glb_cand[e];
            w_next = glb_chc[e];
        }
    };

    // One candidate-phase step k reading its draws at lnbuf[4jG + r] and the
    // row loaded ahead for the current city; `mid` runs before the row's
    // first use (independent work that fills the loads' latency).
    auto cand_step = [&](int k, int j, auto&& mid) {
        const uint32_t node = node_next;
        const float w = w_next;
        mid();
        const float lnu = lds_ln[4 * j * G + ln_lane];
        const uint32_t live = tabu.live(node);
        float key = lnu * w;  // (w holds 1 / choice_info)
        asm volatile("" : "+v"(key));
        // ln(u) < 0 and w >= 0 give a key with the sign bit set (a negative
        // number, -0 or -inf), whose order code is ~bits
        const uint32_t code = ~__float_as_uint(key) & live & lane_ok;
        const uint32_t best = wave_max_u32<kRows>(code);
        uint32_t next = kNone;
        if (best != 0u) {
            const uint64_t tied = __ballot(code == best);
            const int first = (int)__builtin_ctzll(tied);
            next = (uint32_t)__builtin_amdgcn_readlane((int)node, first);
            if (__builtin_expect(first != 63 - (int)__builtin_clzll(tied), 0))
                next = wave_min_u32<kRows>(code == best ? node : kNone);
        }
        if (__builtin_expect(next == kNone, 0)) next = fallback(k);
        load_row((int)next);
        advance(next, k);
    };

    // after the steps before ke: at the end of a 64-step chunk or of the
    // tour, store the chunk's cities and add the lengths of the edges into them
    auto flush = [&](int ke) {
        if ((ke & 63) == 0 || ke == n) {
            // steps c0 .. ke - 1; lane l holds step c0 + l
            const int c0 = (ke - 1) & ~63;
            const int last = ke - 1 - c0;
            const uint32_t prev = __shfl_up(tbuf, 1);
            if (lane <= last) {
                tour_out[c0 + lane] = (uint16_t)tbuf;
                // edge entering step c0 + l (none for step 0)
                const uint32_t from = lane == 0 ? prev_last : prev;
                if (c0 + lane > 0) len += dist[(size_t)from * n + tbuf];
            }
            prev_last = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, last);
        }
    };

    // the draws of the group of steps k0 .. k0 + S - 1, all at once
    auto draws_now = [&](int k0) {
        const Words4 b = draw_block(seed, it, (uint32_t)ant, (uint32_t)(k0 + (lane >> gsh)),
                                    (uint32_t)(4 * (lane & (G - 1))));
        float4 lv;
        lv.x = log_u01(u01(b.w[0]));
        lv.y = log_u01(u01(b.w[1]));
        lv.z = log_u01(u01(b.w[2]));
        lv.w = log_u01(u01(b.w[3]));
        *reinterpret_cast<float4*>(lnbuf + 4 * lane) = lv;
    };

    // steps kb .. ke - 1 of the group starting at k0 (draws in place)
    auto steps_plain = [&](int k0, int kb, int ke) {
        for (int k = kb; k < ke; ++k) cand_step(k, k - k0, [] {});
    };

    if (cl == 0) {
        for (int k = 1; k < n; ++k) {
            advance(fallback(k), k);
            flush(k + 1);
        }
    } else if constexpr (kG > 0 && kHelp) {
        // draws from the helper wave: group g in buffer g & 1
        const LdsPtr<const float> buf0 = (LdsPtr<const float>)lnbuf;
        const LdsPtr<const float> buf1 = (LdsPtr<const float>)reinterpret_cast<float*>(help);
        constexpr int S = kWave / kG;
        load_row(cur);
        int g = 0;
        for (int k0 = 0; k0 < n; k0 += S, ++g) {
            if (!bad_help) bad_help = !wait_count(&hl->made, g + 1);  // (after one timeout, no more waits)
            lds_ln = (g & 1) ? buf1 : buf0;
            const int ke = k0 + S < n ? k0 + S : n;
            steps_plain(k0, k0 > 0 ? k0 : 1, ke);
            lds_put(&hl->read, g + 1);  // after the group's last read of its buffer
            flush(ke);
        }
        lds_put(&hl->stop, 1);
    } else if constexpr (kG > 0) {
        load_row(cur);
        // Draws computed one group ahead, spread over the steps of the group
        // before in seven pieces (three of Philox rounds, the last round with
        // the first logarithm, one logarithm each) that fill the latency of
        // the steps' row loads, and stored after that group's last read.
        constexpr int S = kWave / kG;
        static_assert(S == 8 || S == 16, "pieces are laid out for 8 or 16 steps a group");
        const uint32_t k0s = (uint32_t)seed, k1s = (uint32_t)(seed >> 32);
        draws_now(0);
        steps_plain(0, 1, S < n ? S : n);
        flush(S < n ? S : n);
        if (S < n) draws_now(S);
        int k0 = S;
        for (; k0 + S <= n; k0 += S) {
            Words4 c;
            float lv[4];
            const int kn = k0 + S;  // the group whose draws are computed here
#pragma unroll
            for (int j = 0; j < S; ++j) {
                // piece q of the next group's draws runs at step j = q * S / 8
                auto piece = [&] {
                    if (j * 8 % S != 0) return;
                    const int q = j * 8 / S;
                    // (each piece's results pass through an empty asm in this
                    // step, which keeps the compiler from sinking the piece to
                    // the end of the group, where its results are stored)
                    if (q == 0) {
                        c = Words4{{(uint32_t)(lane & (kG - 1)) | ((uint32_t)(kn + (lane >> gsh)) << 16),
                                    (uint32_t)ant, it, 0u}};
                        philox_rounds<0, 3>(c, k0s, k1s);
                    } else if (q == 1) {
                        philox_rounds<3, 6>(c, k0s, k1s);
                    } else if (q == 2) {
                        philox_rounds<6, 9>(c, k0s, k1s);
                    } else if (q == 3) {
                        philox_rounds<9, 10>(c, k0s, k1s);
                        lv[0] = log_u01(u01(c.w[0]));
                        asm volatile("" : "+v"(lv[0]));
                    } else if (q < 7) {
                        lv[q - 3] = log_u01(u01(c.w[q - 3]));
                        asm volatile("" : "+v"(lv[q - 3]));
                    }
                    if (q < 4) asm volatile("" : "+v"(c.w[0]), "+v"(c.w[1]), "+v"(c.w[2]), "+v"(c.w[3]));
                };
                cand_step(k0 + j, j, piece);
            }
            // after the group's last read of the buffer
            *reinterpret_cast<float4*>(lnbuf + 4 * lane) = make_float4(lv[0], lv[1], lv[2], lv[3]);
            flush(k0 + S);
        }
        if (k0 < n) {
            steps_plain(k0, k0, n);
            flush(n);
        }
    } else {
        load_row(cur);
        for (int k0 = 0; k0 < n; k0 += S) {
            draws_now(k0);
            const int ke = k0 + S < n ? k0 + S : n;
            steps_plain(k0, k0 > 0 ? k0 : 1, ke);
            flush(ke);
        }
    }
    if constexpr (kWide) wide_lead_end(wl, lane);
    if (bad && lane == 0) atomicOr(&vw.state->flags, 8u);
    if (bad_help && lane == 0) atomicOr(&vw.state->flags, 32u);
    if (lane == 0) len += dist[(size_t)cur * n + start];  // closing edge
    len = wave_sum_i64(len);
    if (lane == 0) {
        vw.lengths[ant] = len;
        vw.fallback[ant] = fb_steps;
        vw.fallback[s.ants + ant] = fb_nodes;
    }
}

// Per-half wave64 reductions for two ants per wave (lanes 0-31: first ant,
// 32-63: second): the maximum (minimum) of each half, as two scalars.
__device__ __forceinline__ void half_max_u32(uint32_t x, uint32_t& lo, uint32_t& hi) {
    x = max(x, dpp<0xB1>(x));
    x = max(x, dpp<0x4E>(x));
    x = max(x, dpp<0x141>(x));
    x = max(x, dpp<0x140>(x));
    lo = max((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    hi = max((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
}
__device__ __forceinline__ void half_min_u32(uint32_t x, uint32_t& lo, uint32_t& hi) {
    x = min(x, dpp<0xB1>(x));
    x = min(x, dpp<0x4E>(x));
    x = min(x, dpp<0x141>(x));
    x = min(x, dpp<0x140>(x));
    lo = min((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    hi = min((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
}

// The all-node fallback of one ant (whole wave), as in construct_ant.
template <int kTabu, int kPher, class Tabu>
__device__ uint32_t fallback_step(const Views& vw, const Shape& s, uint32_t it, uint32_t ant, uint32_t cur, int k,
                                  const Tabu& tabu, uint8_t* region, float tmin_a, int lane) {
    const int n = s.n;
    if constexpr (kPher == MMAS_PHER_DENSE) {
        const DenseFactor wt{vw.choice_inv + (size_t)cur * n};
        if constexpr (kTabu == MMAS_TABU_BITMASK) {
            uint16_t* ulist = reinterpret_cast<uint16_t*>(region + kDrawBytes + kScratchBytes + align16(4 * ((n + 31) / 32)));
            return fallback_bitmask(tabu, n, ulist, list_cap(s), wt, s.cl, s.seed, it, ant, (uint32_t)k, lane);
        } else {
            return fallback_list(tabu.list(), tabu.L, wt, s.cl, s.seed, it, ant, (uint32_t)k, lane);
        }
    } else {
        const CandFactor wt{vw.dist + (size_t)cur * n, tmin_a, s.beta};
        if constexpr (kTabu == MMAS_TABU_BITMASK) {
            uint16_t* ulist = reinterpret_cast<uint16_t*>(region + kDrawBytes + kScratchBytes + align16(4 * ((n + 31) / 32)));
            return fallback_bitmask(tabu, n, ulist, list_cap(s), wt, s.cl, s.seed, it, ant, (uint32_t)k, lane);
        } else {
            return fallback_list(tabu.list(), tabu.L, wt, s.cl, s.seed, it, ant, (uint32_t)k, lane);
        }
    }
}

// The visited test of a lane's candidate in a wave serving two ants: lane
// half h reads the tabu of its own ant (~0 if unvisited, else 0).
__device__ __forceinline__ uint32_t live_pair(const BitmaskTabu& a, const BitmaskTabu& b, int h, uint32_t v) {
    const uint32_t* bits = h ? b.bits : a.bits;
    return __builtin_amdgcn_ubfe(bits[v >> 5], v, 1u) - 1u;
}
__device__ __forceinline__ uint32_t live_pair(const CompactTabu& a, const CompactTabu& b, int h, uint32_t v) {
    const uint16_t* e = h ? b.entries : a.entries;
    return e[v] > v ? 0u : ~0u;
}
__device__ __forceinline__ uint32_t live_pair(const ListTabu& a, const ListTabu& b, int h, uint32_t v) {
    const uint16_t* idx = h ? b.idx : a.idx;
    const int L = h ? b.L : a.L;
    return (int)idx[v] >= L ? 0u : ~0u;
}

// Two ants per wave64 (1 <= cl <= 32): lanes 0-31 serve ant `ant0`, lanes
// 32-63 ant `ant0 + 1` (absent if !hasB). Both take their candidate steps
// together: lane 32h + r holds rank r of ant h's current row, the keys and
// the per-half argmax are those of construct_ant. A step in which an ant has
// no unvisited candidate runs that ant's fallback on the whole wave. Same
// draws, same arithmetic, same tours as one ant per wave. Laid out like the
// single colony's step: both current cities wave-uniform, draws generated
// once per group of steps, the visited test folded into the key code.
template <int kTabu, int kPher>
__device__ void construct_pair(const Views& vw, const Shape& s, uint32_t it, int ant0, bool hasB, int lane,
                               uint8_t* regA, uint8_t* regB, const uint16_t* tcand, const float* tchc, int R) {
    using Tabu = typename TabuOf<kTabu>::type;
    const int n = s.n, cl = s.cl;
    const uint64_t seed = s.seed;
    const int h = lane >> 5, hl = lane & 31;
    const uint32_t antA = (uint32_t)ant0, antB = (uint32_t)ant0 + 1u;
    const uint32_t my_ant = h ? antB : antA;

    Tabu tabA, tabB;
    tabA.init(regA + kDrawBytes + kScratchBytes, n, lane);
    tabB.init(regB + kDrawBytes + kScratchBytes, n, lane);
    float* lnbuf = reinterpret_cast<float*>(h ? regB : regA);

    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    const LdsPtr<const uint16_t> lds_cand = (LdsPtr<const uint16_t>)tcand;
    const LdsPtr<const float> lds_chc = (LdsPtr<const float>)tchc;
    const GlbPtr<const uint16_t> glb_cand = (GlbPtr<const uint16_t>)vw.cand;
    const GlbPtr<const float> glb_chc = (GlbPtr<const float>)vw.chc_inv;  // reciprocals

    // start cities: floor(x * n / 2^32) of draw (step 0, slot 0) of each ant
    const uint32_t x0 = draw_block(seed, it, my_ant, 0u, 0u).w[0];
    const uint32_t st_l = (uint32_t)(((uint64_t)x0 * (uint64_t)n) >> 32);
    const int startA = __builtin_amdgcn_readlane((int)st_l, 0);
    const int startB = __builtin_amdgcn_readlane((int)st_l, 32);
    tabA.mark((uint32_t)startA, lane);
    if (hasB) tabB.mark((uint32_t)startB, lane ^ 32);

    // draws ahead, S = 32/G steps at a time, each half for its own ant
    const int gsh = cl <= 4 ? 0 : cl <= 8 ? 1 : cl <= 16 ? 2 : 3;
    const int G = 1 << gsh;
    const int S = 32 >> gsh;
    const int lr = hl < cl ? hl : cl - 1;
    const uint32_t lane_ok = ((hl < cl) & (h == 0 || hasB)) ? ~0u : 0u;
    const int ln_lane = hl & (4 * G - 1);

    uint16_t* tour_out = vw.tours + (size_t)my_ant * n;
    const int32_t* dist = vw.dist;
    const bool writer = h == 0 || hasB;
    uint32_t tbuf = (uint32_t)(h ? startB : startA);  // lane 32h + (k & 31) holds the city of step k
    uint32_t prev_last = 0;
    int64_t len = 0;
    int64_t fbA_steps = 0, fbA_nodes = 0, fbB_steps = 0, fbB_nodes = 0;
    int curA = startA, curB = startB;
    bool bad = false;

    for (int k0 = 0; k0 < n; k0 += S) {
        {
            const Words4 b = draw_block(seed, it, my_ant, (uint32_t)(k0 + (hl >> gsh)), (uint32_t)(4 * (hl & (G - 1))));
            float4 lv;
            lv.x = log_u01(u01(b.w[0]));
            lv.y = log_u01(u01(b.w[1]));
            lv.z = log_u01(u01(b.w[2]));
            lv.w = log_u01(u01(b.w[3]));
            *reinterpret_cast<float4*>(lnbuf + 4 * hl) = lv;
        }
        const int kb = k0 > 0 ? k0 : 1;
        const int ke = k0 + S < n ? k0 + S : n;
        for (int k = kb; k < ke; ++k) {
            const int cur_l = h ? curB : curA;
            const int e = cur_l * cl + lr;
            uint32_t node;
            float w;
            if (R == 0) {
                // no table (a wave-uniform test, so no exec-mask bookkeeping)
                node = glb_cand[e];
                w = glb_chc[e];
            } else if (cur_l >= R) {
                node = glb_cand[e];
                w = glb_chc[e];
            } else {
                node = lds_cand[e];
                w = lds_chc[e];
            }
            const float lnu = lnbuf[4 * (k - k0) * G + ln_lane];
            const uint32_t live = live_pair(tabA, tabB, h, node);
            float key = lnu * w;  // (w holds 1 / choice_info)
            asm volatile("" : "+v"(key));
            // ln(u) < 0 and w >= 0: the key's sign bit is set, its order code is ~bits
            const uint32_t code = ~__float_as_uint(key) & live & lane_ok;
            uint32_t bestA, bestB;
            half_max_u32(code, bestA, bestB);
            const uint32_t best_l = h ? bestB : bestA;
            const uint64_t tied = __ballot(code == best_l);
            const uint32_t tA = (uint32_t)tied, tB = (uint32_t)(tied >> 32);
            uint32_t nextA = kNone, nextB = kNone;
            if (bestA) nextA = (uint32_t)__builtin_amdgcn_readlane((int)node, __builtin_ctz(tA));
            if (bestB) nextB = (uint32_t)__builtin_amdgcn_readlane((int)node, 32 + __builtin_ctz(tB));
            if (__builtin_expect(((tA & (tA - 1)) | (tB & (tB - 1))) != 0, 0)) {
                uint32_t mA, mB;
                half_min_u32(((tied >> lane) & 1ull) ? node : kNone, mA, mB);
                if (bestA) nextA = mA;
                if (bestB) nextB = mB;
            }
            if (__builtin_expect(nextA == kNone, 0)) {
                fbA_steps += 1;
                fbA_nodes += n - k;
                nextA = (uint32_t)__builtin_amdgcn_readfirstlane(
                    (int)fallback_step<kTabu, kPher>(vw, s, it, antA, (uint32_t)curA, k, tabA, regA, tmin_a, lane));
            }
            if (!hasB) {
                nextB = (uint32_t)curB;  // an absent second ant stays at its (valid) start city
            } else if (__builtin_expect(nextB == kNone, 0)) {
                fbB_steps += 1;
                fbB_nodes += n - k;
                nextB = (uint32_t)__builtin_amdgcn_readfirstlane(
                    (int)fallback_step<kTabu, kPher>(vw, s, it, antB, (uint32_t)curB, k, tabB, regB, tmin_a, lane));
            }
            // no city is unreachable with a validated instance; were it not,
            // report it after the tour and go on with city 0 (the tour is void)
            bad |= (nextA >= (uint32_t)n) | (nextB >= (uint32_t)n);
            nextA = nextA < (uint32_t)n ? nextA : 0u;
            nextB = nextB < (uint32_t)n ? nextB : 0u;
            if constexpr (kTabu == MMAS_TABU_BITMASK) {
                // both marks in one LDS OR issued by every lane: lane 0 sets
                // A's bit, lane 32 B's (when B is there), the others OR zero
                // into their own word of the draw buffer
                const uint32_t nx = h ? nextB : nextA;
                const bool setter = hl == 0 && (h == 0 || hasB);
                uint32_t* word = setter ? (h ? tabB.bits : tabA.bits) + (nx >> 5)
                                        : reinterpret_cast<uint32_t*>(lnbuf) + hl;
                atomicOr(word, setter ? 1u << (nx & 31u) : 0u);
            } else {
                tabA.mark(nextA, lane);
                if (hasB) tabB.mark(nextB, lane ^ 32);
            }
            if (hl == (k & 31)) tbuf = h ? nextB : nextA;
            curA = __builtin_amdgcn_readfirstlane((int)nextA);
            curB = __builtin_amdgcn_readfirstlane((int)nextB);
        }
        if ((ke & 31) == 0 || ke == n) {
            // flush steps c0 .. ke - 1; lane 32h + l holds step c0 + l of ant h
            const int c0 = (ke - 1) & ~31;
            const int last = ke - 1 - c0;
            const uint32_t prev = __shfl_up(tbuf, 1);
            if (hl <= last && writer) {
                tour_out[c0 + hl] = (uint16_t)tbuf;
                const uint32_t from = hl == 0 ? prev_last : prev;
                if (c0 + hl > 0) len += dist[(size_t)from * n + tbuf];
            }
            const uint32_t plA = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, last);
            const uint32_t plB = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, 32 + last);
            prev_last = h ? plB : plA;
        }
    }
    if (bad && lane == 0) atomicOr(&vw.state->flags, 8u);
    if (lane == 0) len += dist[(size_t)curA * n + startA];  // closing edges
    if (lane == 32 && hasB) len += dist[(size_t)curB * n + startB];
    for (int o = 16; o >= 1; o >>= 1) len += __shfl_xor(len, o);
    if (lane == 0) {
        vw.lengths[antA] = len;
        vw.fallback[antA] = fbA_steps;
        vw.fallback[s.ants + antA] = fbA_nodes;
    }
    if (lane == 32 && hasB) {
        vw.lengths[antB] = len;
        vw.fallback[antB] = fbB_steps;
        vw.fallback[s.ants + antB] = fbB_nodes;
    }
}

// kRows: 16-lane rows the argmax of a one-ant-per-wave step reduces (2 for
// cl <= 32, else 4); kG: 4-slot draw groups per step when fixed (4 for
// 9 <= cl <= 16, 8 for 17 <= cl <= 32: the draws are then pipelined), else 0.
// Both unused with two ants per wave. kHelp (one ant per wave, kG > 0): the
// workgroup has a draw helper wave per ant (waves apb .. 2 apb - 1 for the
// ants of waves 0 .. apb - 1); each region ends with the helper's part.
template <int kTabu, int kPher, bool kPair, int kRows = 4, int kG = 0, bool kHelp = false>
__global__ __launch_bounds__(1024) void k_construct(Views vw, Shape s, uint32_t it, int ants_per_block, Lds lds) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int R = lds.rows;
    uint16_t* tcand = reinterpret_cast<uint16_t*>(smem);
    float* tchc = reinterpret_cast<float*>(smem + align16(R * s.cl * 2));
    uint8_t* regions = smem + lds.table_bytes;
    if (R > 0) stage_table(vw, s.cl, R, tcand, tchc);
    if constexpr (kHelp) {
        // every ant's HelpLds starts at 0 (three 16-byte stores each)
        if ((int)threadIdx.x < 3 * ants_per_block) {
            const int a = (int)threadIdx.x / 3, q = (int)threadIdx.x % 3;
            *reinterpret_cast<int4*>(regions + (size_t)(a + 1) * lds.per_ant - sizeof(HelpLds) + 16 * q) =
                make_int4(0, 0, 0, 0);
        }
    }
    if (R > 0 || kHelp) __syncthreads();
    const bool helper = kHelp && wave >= ants_per_block;
    const int aw = helper ? wave - ants_per_block : wave;
    const int ant = blockIdx.x * ants_per_block + (kPair ? 2 * aw : aw);
    if (ant >= s.ants) return;  // whole waves leave together
    if constexpr (kHelp) {
        uint8_t* region = regions + (size_t)aw * lds.per_ant;
        uint8_t* help = region + lds.per_ant - kHelpBytes;
        if (helper)
            draw_helper<kTabu, kPher, kG>(vw, s, it, ant, lane, region, help);
        else
            construct_lone<kTabu, kPher, kRows, kG, false, true>(vw, s, it, ant, lane, region, tcand, tchc, R,
                                                                 nullptr, 1, help);
        return;
    }
    if constexpr (kPair)
        construct_pair<kTabu, kPher>(vw, s, it, ant, ant + 1 < s.ants, lane, regions + (size_t)(2 * wave) * lds.per_ant,
                                     regions + (size_t)(2 * wave + 1) * lds.per_ant, tcand, tchc, R);
    else
        construct_lone<kTabu, kPher, kRows, kG>(vw, s, it, ant, lane, regions + (size_t)wave * lds.per_ant, tcand,
                                                tchc, R);
}

// One ant per workgroup of several waves: the leading wave takes the steps
// as in the single colony (construct_lone), the others share its
// fallbacks. LDS: the table part, then the ant's region. kRows, kG as for
// k_construct.
template <int kTabu, int kPher, int kRows = 4, int kG = 0>
__global__ __launch_bounds__(1024) void k_construct_wide(Views vw, Shape s, uint32_t it, Lds lds) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ WideLds wl;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int nw = (int)(blockDim.x >> 6);
    const int R = lds.rows;
    uint16_t* tcand = reinterpret_cast<uint16_t*>(smem);
    float* tchc = reinterpret_cast<float*>(smem + align16(R * s.cl * 2));
    if (R > 0) stage_table(vw, s.cl, R, tcand, tchc);
    __syncthreads();
    uint8_t* region = smem + lds.table_bytes;
    if (wave > 0) {
        wide_helpers<kTabu, kPher>(vw, s, it, (int)blockIdx.x, lane, region, &wl, wave, nw);
        return;
    }
    // the leading wave: the single-colony step, its fallbacks shared
    construct_lone<kTabu, kPher, kRows, kG, true>(vw, s, it, (int)blockIdx.x, lane, region, tcand, tchc, R, &wl, nw);
}

// Without candidate lists, for small instances with SIMDs to spare: a team
// of four waves per ant and no shared tabu. Every step keys all unvisited
// cities (Alg. 4 over all of them, as the fallback does); the cities are
// split by their word in the draw block: wave j takes city 4b + j of every
// block b, so the four waves compute the same Philox blocks (one per lane and
// round) and each keys one word of them. A wave keeps the visited bits of its
// cities in a register (bit r of lane l: city 4 (64 r + l) + j; the bitmask
// tabu held in registers). One barrier a step: each wave posts its best
// (key code, city), and all four read the four and take the same winner, so
// each knows the next city without a second exchange. n <= 1024 (at most four
// rounds of 64 blocks).
template <int kPher>
__global__ __launch_bounds__(256) void k_construct_team(Views vw, Shape s, uint32_t it) {
    __shared__ unsigned long long res[2][4];  // by step parity: each wave's best
    const int lane = threadIdx.x & 63;
    const int j = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));  // word of the block
    const int ant = blockIdx.x;
    const int n = s.n;
    const uint64_t seed = s.seed;
    const int rounds = (((n + 3) >> 2) + kWave - 1) / kWave;  // <= 4
    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    const uint32_t x0 = draw_block(seed, it, (uint32_t)ant, 0u, 0u).w[0];
    const int start = __builtin_amdgcn_readfirstlane((int)(((uint64_t)x0 * (uint64_t)n) >> 32));
    // visited bits; cities past n count as visited
    uint32_t vis = 0u;
#pragma unroll
    for (int r = 0; r < 4; ++r)
        if (r >= rounds || 4 * (kWave * r + lane) + j >= n) vis |= 1u << r;
    auto mark = [&](int c) {
        if ((c & 3) == j && lane == ((c >> 2) & (kWave - 1))) vis |= 1u << (c >> 8);
    };
    mark(start);

    uint16_t* tour_out = vw.tours + (size_t)ant * n;
    const int32_t* dist = vw.dist;
    uint32_t tbuf = (uint32_t)start;  // first wave: lane (k & 63) holds the city of step k
    uint32_t prev_last = 0;
    int64_t len = 0;
    int cur = start;
    for (int k = 1; k < n; ++k) {
        // the factors and visited bits first, then the draws
        float f[4];
        uint32_t v[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int c = 4 * (kWave * r + lane) + j;
            v[r] = c < n ? (uint32_t)c : 0u;
            if (kPher == MMAS_PHER_DENSE)
                f[r] = r < rounds ? vw.choice_inv[(size_t)cur * n + v[r]] : 1.0f;
            else
                f[r] = r < rounds ? 1.0f / (tmin_a * heur_from_dist(dist[(size_t)cur * n + v[r]], s.beta)) : 1.0f;
        }
        uint32_t bcode = 0u, bnode = kNone;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            if (r >= rounds) break;
            const Words4 blk = draw_block(seed, it, (uint32_t)ant, (uint32_t)k, (uint32_t)(4 * (kWave * r + lane)));
            const float key = log_u01(u01(pick_word(blk, (uint32_t)j))) * f[r];
            keep_best(((vis >> r) & 1u) ? 0u : ord_key(key), v[r], bcode, bnode);
        }
        const unsigned long long mine = share_result(bcode, bnode);
        if (lane == 0) res[k & 1][j] = mine;
        __syncthreads();
        // every wave takes the same winner: the largest key code, then the
        // largest ~city (res[k & 1] is written again two steps later, after
        // the next barrier)
        const unsigned long long rr = lane < 4 ? res[k & 1][lane] : 0ull;
        const uint32_t hi = (uint32_t)(rr >> 32), lo = (uint32_t)rr;
        const uint32_t mx = wave_max_u32<2>(hi);
        const uint64_t tied = __ballot(hi == mx && lane < 4);
        uint32_t best_lo;
        if (__popcll(tied) == 1)
            best_lo = (uint32_t)__builtin_amdgcn_readlane((int)lo, __ffsll((unsigned long long)tied) - 1);
        else
            best_lo = wave_max_u32<2>(hi == mx ? lo : 0u);
        const uint32_t next = mx ? ~best_lo : kNone;
        if (next >= (uint32_t)n) {
            // unreachable with a validated instance; every wave leaves
            if (j == 0 && lane == 0) atomicOr(&vw.state->flags, 8u);
            break;
        }
        mark((int)next);
        cur = (int)next;
        if (j == 0) {
            const int slot = k & 63;
            if (lane == slot) tbuf = next;
            if (slot == 63 || k == n - 1) {
                // flush the chunk of steps k0 .. k; lane l holds step k0 + l
                const int k0 = k - slot;
                const uint32_t prev = __shfl_up(tbuf, 1);
                if (lane <= slot) {
                    tour_out[k0 + lane] = (uint16_t)tbuf;
                    const uint32_t from = lane == 0 ? prev_last : prev;
                    if (k0 + lane > 0) len += dist[(size_t)from * n + tbuf];
                }
                prev_last = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, slot);
            }
        }
    }
    if (j != 0) return;
    if (lane == 0) len += dist[(size_t)cur * n + start];  // closing edge
    len = wave_sum_i64(len);
    if (lane == 0) {
        vw.lengths[ant] = len;
        vw.fallback[ant] = n - 1;                                 // every step is a fallback
        vw.fallback[s.ants + ant] = (int64_t)n * (n - 1) / 2;     // over n - k cities at step k
    }
}

// Batched construction: a persistent grid pulls tiles (instance, first ant of
// a group of ants_per_block ants) from a queue ordered by decreasing n. Each
// tile stages as many candidate rows of its instance as fit in the table part
// of LDS, then every wave builds one ant's tour (two with kPair).
template <int kTabu, int kPher, bool kPair>
// (limited to 64 VGPRs, which lets eight waves share a SIMD: the persistent
// batch is bound by instruction issue, and the extra waves hide more latency
// than the few spilled registers cost)
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8))) void k_batch_construct(const BatchItem* __restrict__ items,
                                                          const BatchTile* __restrict__ tiles, int ntiles,
                                                          uint32_t* __restrict__ queue, const uint32_t* __restrict__ it_dev,
                                                          int ants_per_block, int table_bytes, int per_ant) {
    extern __shared__ __align__(16) uint8_t smem[];
    __shared__ int s_tile;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const uint32_t it = *it_dev;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(queue, 1u);
        __syncthreads();
        const int t = s_tile;
        if (t >= ntiles) break;  // every wave of the workgroup leaves here
        const BatchTile tile = tiles[t];
        const Views vw = items[tile.inst].v;
        const Shape s = items[tile.inst].s;
        int R = 0;
        if (s.cl > 0) {
            R = (table_bytes - 16) / (s.cl * 6);
            if (R > s.n) R = s.n;
            while (R > 0 && align16(R * s.cl * 2) + R * s.cl * 4 > table_bytes) --R;
        }
        uint16_t* tcand = reinterpret_cast<uint16_t*>(smem);
        float* tchc = reinterpret_cast<float*>(smem + align16(R * s.cl * 2));
        if (R > 0) stage_table(vw, s.cl, R, tcand, tchc);
        __syncthreads();
        const int ant = tile.ant0 + (kPair ? 2 * wave : wave);
        uint8_t* regions = smem + table_bytes;
        if (ant < s.ants) {
            if constexpr (kPair)
                construct_pair<kTabu, kPher>(vw, s, it, ant, ant + 1 < s.ants, lane,
                                             regions + (size_t)(2 * wave) * per_ant,
                                             regions + (size_t)(2 * wave + 1) * per_ant, tcand, tchc, R);
            else
                construct_ant<kTabu, kPher>(vw, s, it, ant, lane, regions + (size_t)wave * per_ant, tcand, tchc, R);
        }
        __syncthreads();  // the next tile reuses the table part
    }
}

}  // namespace

// Per-device attributes, read once per device (up to 64 devices).
namespace {
constexpr int kMaxDevices = 64;
std::atomic<int> g_lds[kMaxDevices];
std::atomic<int> g_simds[kMaxDevices];
std::atomic<int> g_cus[kMaxDevices];

int device_attr(std::atomic<int>* cache, hipDeviceAttribute_t attr, int scale, int fallback) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return fallback;
    int v = cache[dev].load(std::memory_order_relaxed);
    if (v > 0) return v;
    int a = 0;
    v = hipDeviceGetAttribute(&a, attr, dev) == hipSuccess && a > 0 ? a * scale : fallback;
    cache[dev].store(v, std::memory_order_relaxed);
    return v;
}
}  // namespace

int max_lds_per_block() { return device_attr(g_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, 1, 65536); }

namespace {

// Two ants per wave when asked for and 1 <= cl <= 32 (the candidate row fits
// in a half wave).
bool pair_ok(const Shape& s) { return s.lanes_per_ant == 32 && s.cl >= 1 && s.cl <= 32; }

template <int kTabu, int kPher, bool kPair, int kRows = 4, int kG = 0>
hipError_t launch_t(const Views& v, const Shape& s0, uint32_t it, hipStream_t st) {
    // one colony: a workgroup per four ants rarely shares a CU, so the fallback
    // lists every unvisited city in one pass
    Shape s = s0;
    s.list_cap = s.n;
    // a draw helper wave per ant (one ant per wave with pipelined draws) by
    // default while every ant's wave has a SIMD of its own, which the helper
    // then shares; not with one wave per ant asked for
    const bool help = !kPair && kG > 0 && s.construct_waves == 0 &&
                      s.ants <= device_attr(g_simds, hipDeviceAttributeMultiprocessorCount, 4, 0);
    const int per_ant = (int)construct_lds_per_ant(s) + (help ? (int)kHelpBytes : 0);
    const int budget = max_lds_per_block();
    int apb = s.ants_per_block > 0 ? s.ants_per_block : 4;
    const int step = kPair ? 2 : 1;  // ants per wave
    if (apb < step) apb = step;
    if (help && apb > 8) apb = 8;  // two waves per ant, at most 16 a workgroup
    while (apb > step && per_ant * apb > budget) apb -= step;
    if (per_ant * apb > budget) return hipErrorInvalidValue;
    // as many rows of the candidate table as fit next to the ants' regions;
    // by default only in one workgroup's share of a CU's LDS when the grid
    // needs several per CU (a full table would leave one resident workgroup
    // per CU: 3795 ants at n = 3795 took 8.9 ms instead of 3.5 ms)
    const int blocks = (s.ants + apb - 1) / apb;
    int lds_wg = budget;
    const int cus = device_attr(g_cus, hipDeviceAttributeMultiprocessorCount, 1, 0);
    if (cus > 0 && s.table_rows < 0) {
        const int waves = apb / step * (help ? 2 : 1);
        int per_cu = (blocks + cus - 1) / cus;
        const int most = waves < 32 ? 32 / waves : 1;  // eight waves per SIMD
        if (per_cu > most) per_cu = most;
        if (per_cu > 1) lds_wg = budget / per_cu;
    }
    Lds lds{};
    lds.per_ant = per_ant;
    const int row_bytes = s.cl * 6;
    int rows = 0;
    if (s.cl > 0) {
        rows = (lds_wg - apb * per_ant - 32) / row_bytes;
        if (rows > s.n) rows = s.n;
        if (s.table_rows >= 0 && rows > s.table_rows) rows = s.table_rows;
        while (rows > 0 && align16(rows * s.cl * 2) + align16(rows * s.cl * 4) + apb * per_ant > budget) --rows;
        if (rows < 0) rows = 0;
    }
    lds.rows = rows;
    lds.table_bytes = align16(rows * s.cl * 2) + align16(rows * s.cl * 4);
    const size_t bytes = (size_t)lds.table_bytes + (size_t)apb * per_ant;
    auto kern = k_construct<kTabu, kPher, kPair, kRows, kG>;
    if constexpr (!kPair && kG > 0) {
        if (help) kern = k_construct<kTabu, kPher, false, kRows, kG, true>;
    }
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    kern<<<blocks, 64 * (apb / step) * (help ? 2 : 1), bytes, st>>>(v, s, it, apb, lds);
    return hipGetLastError();
}

// Waves per ant for the construction: the launch option, or (0) a choice by
// where the all-city fallback dominates the step, the only part the helper
// waves share. With n >= 8192 (long fallbacks) and SIMDs to spare: as many
// as the SIMDs left over by one wave per ant allow, a power of two up to 16.
// Without a candidate list at n >= 512: four (the bitmask tabu's cities are
// then gathered by the workgroup, one LDS atomic per wave). Otherwise one:
// the per-step barriers then cost more than the shared fallbacks save
// (measured at n = 198, 1002 and 3795 with and without lists).
int construct_waves(const Shape& s) {
    if (s.construct_waves > 0) return s.construct_waves;
    if (s.n >= 8192) {
        // four SIMDs per compute unit
        const int simds = device_attr(g_simds, hipDeviceAttributeMultiprocessorCount, 4, 0);
        int w = 1;
        while (w < 16 && 2 * w * s.ants <= simds) w *= 2;
        return w;
    }
    if (s.cl == 0 && s.n >= 512) return 4;
    return 1;
}

template <int kTabu, int kPher>
hipError_t launch_wide(const Views& v, const Shape& s, uint32_t it, int waves, hipStream_t st) {
    const int per_ant = (int)wide_lds_per_ant(s);
    const int budget = max_lds_per_block() - (int)sizeof(WideLds) - 64;
    if (per_ant > budget) return hipErrorInvalidValue;
    Lds lds{};
    lds.per_ant = per_ant;
    int rows = 0;
    if (s.cl > 0) {
        rows = (budget - per_ant - 32) / (s.cl * 6);
        if (rows > s.n) rows = s.n;
        if (s.table_rows >= 0 && rows > s.table_rows) rows = s.table_rows;
        while (rows > 0 && align16(rows * s.cl * 2) + align16(rows * s.cl * 4) + per_ant > budget) --rows;
        if (rows < 0) rows = 0;
    }
    lds.rows = rows;
    lds.table_bytes = align16(rows * s.cl * 2) + align16(rows * s.cl * 4);
    const size_t bytes = (size_t)lds.table_bytes + (size_t)per_ant;
    auto kern = s.cl > 16 && s.cl <= 32 ? k_construct_wide<kTabu, kPher, 2, 8>
                : s.cl > 8 && s.cl <= 16 ? k_construct_wide<kTabu, kPher, 2, 4>
                : s.cl <= 32             ? k_construct_wide<kTabu, kPher, 2>
                                         : k_construct_wide<kTabu, kPher, 4>;
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    kern<<<s.ants, 64 * waves, bytes, st>>>(v, s, it, lds);
    return hipGetLastError();
}

// The team kernel (four waves per ant, no list, bitmask tabu, n <= 1024):
// by default, or asked for with four waves per ant. Measured at n = 1002
// with 1002 ants (four waves per SIMD): 2.55 ms against 2.92 ms with four
// waves sharing the fallbacks and 3.06 ms with one wave per ant.
bool team_ok(const Shape& s) {
    if (s.cl != 0 || s.tabu != MMAS_TABU_BITMASK || s.n > 1024 || s.select != MMAS_SELECT_WRS) return false;
    return s.construct_waves == 0 || s.construct_waves == 4;
}

template <int kPher>
hipError_t launch_team(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    k_construct_team<kPher><<<s.ants, 4 * kWave, 0, st>>>(v, s, it);
    return hipGetLastError();
}

template <int kTabu, int kPher>
hipError_t launch_tp(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    if (kTabu == MMAS_TABU_BITMASK && team_ok(s)) return launch_team<kPher>(v, s, it, st);
    if (pair_ok(s)) return launch_t<kTabu, kPher, true>(v, s, it, st);
    const int waves = construct_waves(s);
    if (waves > 1) return launch_wide<kTabu, kPher>(v, s, it, waves, st);
    if (s.cl > 16 && s.cl <= 32) return launch_t<kTabu, kPher, false, 2, 8>(v, s, it, st);
    if (s.cl > 8 && s.cl <= 16) return launch_t<kTabu, kPher, false, 2, 4>(v, s, it, st);
    if (s.cl <= 32) return launch_t<kTabu, kPher, false, 2>(v, s, it, st);
    return launch_t<kTabu, kPher, false, 4>(v, s, it, st);
}

// the persistent batched kernel for a configuration
const void* batch_kernel(int tabu, int pher, bool pair) {
    if (tabu == MMAS_TABU_BITMASK) {
        if (pher == MMAS_PHER_DENSE)
            return pair ? (const void*)k_batch_construct<MMAS_TABU_BITMASK, MMAS_PHER_DENSE, true>
                        : (const void*)k_batch_construct<MMAS_TABU_BITMASK, MMAS_PHER_DENSE, false>;
        return pair ? (const void*)k_batch_construct<MMAS_TABU_BITMASK, MMAS_PHER_CANDIDATES, true>
                    : (const void*)k_batch_construct<MMAS_TABU_BITMASK, MMAS_PHER_CANDIDATES, false>;
    }
    if (tabu == MMAS_TABU_COMPACT) {
        if (pher == MMAS_PHER_DENSE)
            return pair ? (const void*)k_batch_construct<MMAS_TABU_COMPACT, MMAS_PHER_DENSE, true>
                        : (const void*)k_batch_construct<MMAS_TABU_COMPACT, MMAS_PHER_DENSE, false>;
        return pair ? (const void*)k_batch_construct<MMAS_TABU_COMPACT, MMAS_PHER_CANDIDATES, true>
                    : (const void*)k_batch_construct<MMAS_TABU_COMPACT, MMAS_PHER_CANDIDATES, false>;
    }
    if (pher == MMAS_PHER_DENSE)
        return pair ? (const void*)k_batch_construct<MMAS_TABU_LIST, MMAS_PHER_DENSE, true>
                    : (const void*)k_batch_construct<MMAS_TABU_LIST, MMAS_PHER_DENSE, false>;
    return pair ? (const void*)k_batch_construct<MMAS_TABU_LIST, MMAS_PHER_CANDIDATES, true>
                : (const void*)k_batch_construct<MMAS_TABU_LIST, MMAS_PHER_CANDIDATES, false>;
}

}  // namespace

size_t construct_lds_per_ant(const Shape& s) {
    // draws; tabu (bitmask words, or compact entries); for the bitmask, the
    // list of unvisited cities built in a fallback
    const int bits = align16(4 * ((s.n + 31) / 32));
    const int tab = s.tabu == MMAS_TABU_BITMASK ? bits + align16(2 * list_cap(s))
                    : s.tabu == MMAS_TABU_COMPACT ? align16(2 * s.n) : align16(4 * s.n);
    return kDrawBytes + kScratchBytes + tab;
}

size_t wide_lds_per_ant(const Shape& s) {
    // as construct_lds_per_ant, with room to list every unvisited city at once
    const int bits = align16(4 * ((s.n + 31) / 32));
    const int list = align16(2 * s.n);
    const int tab = s.tabu == MMAS_TABU_BITMASK ? bits + list : s.tabu == MMAS_TABU_COMPACT ? list : align16(4 * s.n);
    return kDrawBytes + kScratchBytes + tab;
}

hipError_t launch_batch_construct(const BatchItem* items, const BatchTile* tiles, int ntiles, uint32_t* queue,
                                  const uint32_t* it_dev, int tabu, int pher, int ants_per_block, int lanes_per_ant,
                                  int table_bytes, int per_ant, int grid, hipStream_t st) {
    const size_t bytes = (size_t)table_bytes + (size_t)ants_per_block * per_ant;
    const bool pair = lanes_per_ant == 32;
    const void* kern = batch_kernel(tabu, pher, pair);
    // the LDS limit was raised by batch_construct_grid for this footprint (a
    // graph capture must not need it here)
    void* args[] = {(void*)&items, (void*)&tiles, (void*)&ntiles, (void*)&queue, (void*)&it_dev,
                    (void*)&ants_per_block, (void*)&table_bytes, (void*)&per_ant};
    return hipLaunchKernel(kern, dim3(grid), dim3(64 * (pair ? ants_per_block / 2 : ants_per_block)), args, bytes, st);
}

int batch_construct_grid(int tabu, int pher, int ants_per_block, int lanes_per_ant, int lds_bytes) {
    const bool pair = lanes_per_ant == 32;
    const void* kern = batch_kernel(tabu, pher, pair);
    if (lds_bytes > 64 * 1024 &&
        hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();  // do not leave the error for the next launch check
        return 0;
    }
    int per_cu = 0, dev = 0, cus = 0;
    const int threads = 64 * (pair ? ants_per_block / 2 : ants_per_block);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, threads, lds_bytes) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return 0;
    return per_cu * cus;
}

namespace {

// ---- the parallel roulette wheel (Sec. 4.2.1), the paper's baseline ---------

// Inclusive prefix sum of FP32 values over the wave: a log-step scan within
// each row of 16 (lanes below the shift add 0), then every row adds the
// totals of the rows before it, in a fixed order.
__device__ __forceinline__ float wave_scan_f32(float x, int lane) {
    x = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x111, 0xF, 0xF, false));
    x = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x112, 0xF, 0xF, false));
    x = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x114, 0xF, 0xF, false));
    x = x + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x118, 0xF, 0xF, false));
    const float t0 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 15));
    const float t1 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 31));
    const float t2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 47));
    const int row = lane >> 4;
    float add = 0.0f;
    if (row >= 1) add = t0;
    if (row >= 2) add = add + t1;
    if (row >= 3) add = add + t2;
    return x + add;
}

// The wheel over entries 0 .. m-1 of `list` with weights wt(list[i]): 64
// chunks of ceil(len/64) a stage (chunk sums left to right), their prefix
// sums, target u times the total, the first chunk whose prefix exceeds it
// (the last with a positive sum if rounding leaves none), the target less the
// prefix before it, and again inside that chunk until a chunk is one entry.
// Returns the entry; 0 if every weight is 0.
template <class W>
__device__ int prwm_list(const uint16_t* list, int m, const W& wt, float u, int lane) {
    int lo = 0, len = m;
    float target = 0.0f;
    bool first = true;
    for (;;) {
        const int c = (len + 63) >> 6;
        float a = 0.0f;
        const int q1 = (lane + 1) * c < len ? (lane + 1) * c : len;
        for (int q = lane * c; q < q1; ++q) a = a + wt((uint32_t)list[lo + q]);
        const float P = wave_scan_f32(a, lane);
        if (first) {
            const uint64_t pos = __ballot(a > 0.0f);
            if (pos == 0ull) return 0;
            target = u * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P), 63));
            first = false;
        }
        const uint64_t over = __ballot((P > target) & (a > 0.0f));
        const uint64_t pos = __ballot(a > 0.0f);
        const int win = over ? (int)__builtin_ctzll(over) : pos ? 63 - (int)__builtin_clzll(pos) : 0;
        if (win > 0) target = target - __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P), win - 1));
        lo += win * c;
        if (c == 1) return lo;
        len = len - win * c < c ? len - win * c : c;
    }
}

// One ant per wave, bitmask tabu and the full list of unvisited cities in
// LDS (the wheel's chunks follow the ascending city order), rows read from
// global memory. One draw per step (slot 0).
template <int kPher>
__global__ __launch_bounds__(256) void k_construct_prwm(Views vw, Shape s, uint32_t it, int ants_per_block,
                                                        int per_ant) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int ant = blockIdx.x * ants_per_block + wave;
    if (ant >= s.ants) return;
    const int n = s.n, cl = s.cl;
    uint8_t* region = smem + (size_t)wave * per_ant;
    BitmaskTabu tabu;
    tabu.init(region, n, lane);
    uint16_t* ulist = reinterpret_cast<uint16_t*>(region + align16(4 * ((n + 31) / 32)));
    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);
    const uint32_t x0 = draw_block(s.seed, it, (uint32_t)ant, 0u, 0u).w[0];
    const uint32_t start = (uint32_t)(((uint64_t)x0 * (uint64_t)n) >> 32);
    tabu.mark(start, lane);
    uint16_t* tour_out = vw.tours + (size_t)ant * n;
    const int32_t* dist = vw.dist;
    uint32_t tbuf = start, prev_last = 0, cur = start;
    int64_t len = 0, fb_steps = 0, fb_nodes = 0;
    for (int k = 1; k < n; ++k) {
        const float u = u01(draw_block(s.seed, it, (uint32_t)ant, (uint32_t)k, 0u).w[0]);
        uint32_t next = kNone;
        if (cl > 0) {
            const int e = (int)cur * cl + (lane < cl ? lane : cl - 1);
            const uint32_t node = vw.cand[e];
            const float w = vw.chc[e];
            const float a = ((lane < cl) & !tabu.visited(node)) ? w : 0.0f;
            const uint64_t pos = __ballot(a > 0.0f);
            if (pos) {
                const float P = wave_scan_f32(a, lane);
                const float target = u * __int_as_float(__builtin_amdgcn_readlane(__float_as_int(P), 63));
                const uint64_t over = __ballot((P > target) & (a > 0.0f));
                const int win = over ? (int)__builtin_ctzll(over) : 63 - (int)__builtin_clzll(pos);
                next = (uint32_t)__builtin_amdgcn_readlane((int)node, win);
            }
        }
        if (next == kNone) {
            fb_steps += 1;
            fb_nodes += n - k;
            // every unvisited city, ascending (one pass: the list has room for n)
            const int words = (n + 31) >> 5;
            int L = 0;
            for (int w0 = 0; w0 < words; w0 += kWave) {
                const int wi = w0 + lane;
                uint32_t fr = 0u;
                if (wi < words) {
                    fr = ~tabu.bits[wi];
                    if (wi == words - 1 && (n & 31)) fr &= (1u << (n & 31)) - 1u;
                }
                const int cnt = __popc(fr);
                const int incl = wave_incl_scan(cnt, lane);
                int p = L + incl - cnt;
                while (fr) {
                    const int b = __ffs(fr) - 1;
                    fr &= fr - 1u;
                    ulist[p++] = (uint16_t)(wi * 32 + b);
                }
                L += __builtin_amdgcn_readlane(incl, 63);
            }
            int pick;
            if constexpr (kPher == MMAS_PHER_DENSE) {
                const DenseWeight wt{vw.choice + (size_t)cur * n};
                pick = prwm_list(ulist, L, wt, u, lane);
            } else {
                const CandWeight wt{dist + (size_t)cur * n, tmin_a, s.beta};
                pick = prwm_list(ulist, L, wt, u, lane);
            }
            next = L > 0 ? (uint32_t)ulist[pick] : kNone;
        }
        next = (uint32_t)__builtin_amdgcn_readfirstlane((int)next);
        if (next >= (uint32_t)n) {
            if (lane == 0) atomicOr(&vw.state->flags, 8u);
            return;
        }
        tabu.mark(next, lane);
        const int slot = k & 63;
        if (lane == slot) tbuf = next;
        cur = next;
        if (slot == 63 || k == n - 1) {
            const int k0 = k - slot;
            const uint32_t prev = __shfl_up(tbuf, 1);
            if (lane <= slot) {
                tour_out[k0 + lane] = (uint16_t)tbuf;
                const uint32_t from = lane == 0 ? prev_last : prev;
                if (k0 + lane > 0) len += dist[(size_t)from * n + tbuf];
            }
            prev_last = (uint32_t)__builtin_amdgcn_readlane((int)tbuf, slot);
        }
    }
    if (lane == 0) len += dist[(size_t)cur * n + start];
    len = wave_sum_i64(len);
    if (lane == 0) {
        vw.lengths[ant] = len;
        vw.fallback[ant] = fb_steps;
        vw.fallback[s.ants + ant] = fb_nodes;
    }
}

template <int kPher>
hipError_t launch_prwm(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    const int per_ant = align16(4 * ((s.n + 31) / 32)) + align16(2 * s.n);
    const int budget = max_lds_per_block();
    int apb = 4;
    while (apb > 1 && apb * per_ant > budget) --apb;
    if (apb * per_ant > budget) return hipErrorInvalidValue;
    const size_t bytes = (size_t)apb * per_ant;
    auto kern = k_construct_prwm<kPher>;
    if (bytes > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
        if (e != hipSuccess) return e;
    }
    kern<<<(s.ants + apb - 1) / apb, 64 * apb, bytes, st>>>(v, s, it, apb, per_ant);
    return hipGetLastError();
}

// One wave marks marks[0 .. count) in a fresh tabu of n cities, in order, then
// writes visited[v] for every city, the tabu's cells (bitmask: its 32-bit
// words as pairs of 16-bit halves, low first; compact: entries[0 .. n); list:
// unv[0 .. n) then idx[0 .. n)) and the unvisited count (-1 if a mark was out
// of range or already visited: the marking stops there).
template <int kTabu>
__global__ __launch_bounds__(64) void k_eval_tabu(int n, const int32_t* __restrict__ marks, int count,
                                                  uint8_t* __restrict__ visited, uint16_t* __restrict__ state,
                                                  int32_t* __restrict__ left) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x;
    typename TabuOf<kTabu>::type tabu;
    tabu.init(smem, n, lane);
    int bad = 0;
    for (int q = 0; q < count; ++q) {
        const int u = __builtin_amdgcn_readfirstlane(marks[q]);
        if (u < 0 || u >= n || tabu.visited((uint32_t)u)) {
            bad = 1;
            break;
        }
        tabu.mark((uint32_t)u, lane);
    }
    for (int v = lane; v < n; v += kWave) visited[v] = tabu.visited((uint32_t)v) ? 1 : 0;
    if constexpr (kTabu == MMAS_TABU_BITMASK) {
        for (int w = lane; w < (n + 31) / 32; w += kWave) {
            state[2 * w] = (uint16_t)(tabu.bits[w] & 0xFFFFu);
            state[2 * w + 1] = (uint16_t)(tabu.bits[w] >> 16);
        }
    } else if constexpr (kTabu == MMAS_TABU_COMPACT) {
        for (int v = lane; v < n; v += kWave) state[v] = tabu.entries[v];
    } else {
        for (int v = lane; v < n; v += kWave) {
            state[v] = tabu.unv[v];
            state[n + v] = tabu.idx[v];
        }
    }
    if (lane == 0) *left = bad ? -1 : n - count;
}

}  // namespace

hipError_t launch_eval_tabu(int tabu, int n, const int32_t* marks, int count, uint8_t* visited, uint16_t* state,
                            int32_t* left, hipStream_t st) {
    const size_t bytes = tabu == MMAS_TABU_BITMASK ? (size_t)align16(4 * ((n + 31) / 32))
                                                   : (size_t)align16((tabu == MMAS_TABU_COMPACT ? 2 : 4) * n);
    if (tabu == MMAS_TABU_BITMASK)
        k_eval_tabu<MMAS_TABU_BITMASK><<<1, kWave, bytes, st>>>(n, marks, count, visited, state, left);
    else if (tabu == MMAS_TABU_COMPACT)
        k_eval_tabu<MMAS_TABU_COMPACT><<<1, kWave, bytes, st>>>(n, marks, count, visited, state, left);
    else
        k_eval_tabu<MMAS_TABU_LIST><<<1, kWave, bytes, st>>>(n, marks, count, visited, state, left);
    return hipGetLastError();
}

hipError_t launch_construct(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    if (s.select == MMAS_SELECT_PRWM)
        return s.pher == MMAS_PHER_DENSE ? launch_prwm<MMAS_PHER_DENSE>(v, s, it, st)
                                         : launch_prwm<MMAS_PHER_CANDIDATES>(v, s, it, st);
    if (s.tabu == MMAS_TABU_BITMASK) {
        return s.pher == MMAS_PHER_DENSE ? launch_tp<MMAS_TABU_BITMASK, MMAS_PHER_DENSE>(v, s, it, st)
                                         : launch_tp<MMAS_TABU_BITMASK, MMAS_PHER_CANDIDATES>(v, s, it, st);
    }
    if (s.tabu == MMAS_TABU_COMPACT) {
        return s.pher == MMAS_PHER_DENSE ? launch_tp<MMAS_TABU_COMPACT, MMAS_PHER_DENSE>(v, s, it, st)
                                         : launch_tp<MMAS_TABU_COMPACT, MMAS_PHER_CANDIDATES>(v, s, it, st);
    }
    return s.pher == MMAS_PHER_DENSE ? launch_tp<MMAS_TABU_LIST, MMAS_PHER_DENSE>(v, s, it, st)
                                     : launch_tp<MMAS_TABU_LIST, MMAS_PHER_CANDIDATES>(v, s, it, st);
}

}  // namespace mmas
