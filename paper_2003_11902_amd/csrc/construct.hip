// Tour construction (the inner loops of Alg. 1): one ant per wave64.
//
// Each step selects the next city by weighted reservoir sampling (Alg. 4):
// every eligible city v draws u and gets the key ln(u) / w(cur, v); the wave
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
#include "device.hpp"
#include "internal.hpp"

namespace mmas {
namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;

// ---- tabu variants ---------------------------------------------------------

struct BitmaskTabu {
    uint32_t* bits;
    __device__ void init(uint8_t* lds, int n, int lane) {
        bits = reinterpret_cast<uint32_t*>(lds);
        const int words = (n + 31) >> 5;
        for (int w = lane; w < words; w += kWave) bits[w] = 0u;
    }
    __device__ __forceinline__ bool visited(uint32_t v) const { return (bits[v >> 5] >> (v & 31u)) & 1u; }
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
    __device__ void init(uint8_t* lds, int n_, int lane) {
        entries = reinterpret_cast<uint16_t*>(lds);
        n = n_;
        L = n_;
        for (int i = lane; i < n_; i += kWave) entries[i] = (uint16_t)i;
    }
    __device__ __forceinline__ bool visited(uint32_t v) const { return entries[v] > v; }
    __device__ __forceinline__ void mark(uint32_t u, int lane) {
        // every lane reads the same cells; lane 0 writes
        const int iu = entries[u];  // position of u in the left part
        L = L - 1;
        const int t = entries[L];   // last city of the left part
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

// ---- fallback weights --------------------------------------------------------

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

__device__ __forceinline__ void keep_best(uint32_t code, uint32_t node, uint32_t& bcode, uint32_t& bnode) {
    if (code > bcode || (code == bcode && node < bnode)) {
        bcode = code;
        bnode = node;
    }
}

// All-node fallback over the bitmask: lane l takes the slot groups
// g = cl/4 + l, + 64, ...; group g holds slots 4g..4g+3, i.e. cities
// 4g - cl .. 4g - cl + 3, and one Philox block serves all four.
template <class W>
__device__ uint32_t fallback(const BitmaskTabu& tabu, const W& weight, int n, int cl, uint64_t seed,
                             uint32_t it, uint32_t ant, uint32_t step, int lane) {
    uint32_t bcode = 0u, bnode = kNone;
    const int g0 = cl >> 2, g1 = (cl + n - 1) >> 2;
    for (int g = g0 + lane; g <= g1; g += kWave) {
        const int v0 = 4 * g - cl;
        bool any = false;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = v0 + j;
            any |= (v >= 0 && v < n && !tabu.visited((uint32_t)v));
        }
        if (!any) continue;
        const Words4 blk = draw_block(seed, it, ant, step, (uint32_t)(4 * g));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int v = v0 + j;
            if (v < 0 || v >= n || tabu.visited((uint32_t)v)) continue;
            const float key = log_u01(u01(blk.w[j])) / weight((uint32_t)v);
            keep_best(ord_key(key), (uint32_t)v, bcode, bnode);
        }
    }
    return wave_select(bcode, bnode);
}

// All-node fallback over the compact tabu: the left part lists exactly the
// unvisited cities; each draws its own slot cl + v.
template <class W>
__device__ uint32_t fallback(const CompactTabu& tabu, const W& weight, int /*n*/, int cl, uint64_t seed,
                             uint32_t it, uint32_t ant, uint32_t step, int lane) {
    uint32_t bcode = 0u, bnode = kNone;
    for (int i = lane; i < tabu.L; i += kWave) {
        const uint32_t v = tabu.entries[i];
        const uint32_t slot = (uint32_t)cl + v;
        const Words4 blk = draw_block(seed, it, ant, step, slot);
        const float key = log_u01(u01(pick_word(blk, slot & 3u))) / weight(v);
        keep_best(ord_key(key), v, bcode, bnode);
    }
    return wave_select(bcode, bnode);
}

template <int kTabu, int kPher>
__global__ __launch_bounds__(256) void k_construct(Views vw, Shape s, uint32_t it, int ants_per_block,
                                                   int lds_per_ant) {
    extern __shared__ __align__(16) uint8_t smem[];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ant = blockIdx.x * ants_per_block + wave;
    if (wave >= ants_per_block || ant >= s.ants) return;  // whole waves leave together

    const int n = s.n, cl = s.cl;
    const uint64_t seed = s.seed;
    typename TabuOf<kTabu>::type tabu;
    tabu.init(smem + (size_t)wave * lds_per_ant, n, lane);

    float tmin_a = 0.0f;
    if (kPher == MMAS_PHER_CANDIDATES) tmin_a = powi(vw.state->tau_min, s.alpha);

    // start city: floor(x * n / 2^32) of draw (step 0, slot 0)
    const uint32_t x0 = draw_block(seed, it, (uint32_t)ant, 0u, 0u).w[0];
    const uint32_t start = (uint32_t)(((uint64_t)x0 * (uint64_t)n) >> 32);
    tabu.mark(start, lane);

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
            uint32_t code = 0u, node = kNone;
            if (lane < cl) {
                const size_t e = (size_t)cur * cl + lane;
                node = vw.cand[e];
                const float w = vw.chc[e];
                const Words4 blk = draw_block(seed, it, (uint32_t)ant, (uint32_t)k, (uint32_t)lane);
                const float lnu = log_u01(u01(pick_word(blk, (uint32_t)lane & 3u)));
                if (!tabu.visited(node)) code = ord_key(lnu / w);
            }
            next = wave_select(code, node);
        }
        if (next == kNone) {
            fb_steps += 1;
            fb_nodes += n - k;
            if constexpr (kPher == MMAS_PHER_DENSE) {
                const DenseWeight wt{vw.choice + (size_t)cur * n};
                next = fallback(tabu, wt, n, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
            } else {
                const CandWeight wt{dist + (size_t)cur * n, tmin_a, s.beta};
                next = fallback(tabu, wt, n, cl, seed, it, (uint32_t)ant, (uint32_t)k, lane);
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

template <int kTabu, int kPher>
hipError_t launch_t(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    const size_t per_ant = construct_lds_per_ant(s);
    int apb = 4;
    while (apb > 1 && per_ant * apb > 64 * 1024) --apb;
    const size_t lds = per_ant * apb;
    auto kern = k_construct<kTabu, kPher>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    const int blocks = (s.ants + apb - 1) / apb;
    kern<<<blocks, 64 * apb, lds, st>>>(v, s, it, apb, (int)per_ant);
    return hipGetLastError();
}

}  // namespace

size_t construct_lds_per_ant(const Shape& s) {
    size_t b = s.tabu == MMAS_TABU_BITMASK ? sizeof(uint32_t) * (size_t)((s.n + 31) / 32)
                                           : sizeof(uint16_t) * (size_t)s.n;
    return (b + 15) & ~(size_t)15;
}

hipError_t launch_construct(const Views& v, const Shape& s, uint32_t it, hipStream_t st) {
    if (s.tabu == MMAS_TABU_BITMASK) {
        return s.pher == MMAS_PHER_DENSE ? launch_t<MMAS_TABU_BITMASK, MMAS_PHER_DENSE>(v, s, it, st)
                                         : launch_t<MMAS_TABU_BITMASK, MMAS_PHER_CANDIDATES>(v, s, it, st);
    }
    return s.pher == MMAS_PHER_DENSE ? launch_t<MMAS_TABU_COMPACT, MMAS_PHER_DENSE>(v, s, it, st)
                                     : launch_t<MMAS_TABU_COMPACT, MMAS_PHER_CANDIDATES>(v, s, it, st);
}

}  // namespace mmas
