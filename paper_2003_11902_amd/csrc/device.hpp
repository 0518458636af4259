// Device-side building blocks shared by the kernels of the library:
// counter-based random numbers, the FP32 logarithm used for the reservoir
// keys, the orderable (key, node) encoding and wave64 reductions.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mmas {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11): per round, words 0 and
// 2 are multiplied by two fixed constants; the new counter is
// (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0)); the key is
// bumped by the two Weyl constants after each round.
// ---------------------------------------------------------------------------
struct Words4 {
    uint32_t w[4];
};

// Rounds r0 .. r1 - 1 of Philox4x32-10 on the counter c with the key
// (k0, k1) of round 0 (round r uses k + r times the Weyl constants), so that
// the ten rounds can be spread over several calls.
template <int r0, int r1>
__device__ __forceinline__ void philox_rounds(Words4& c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int round = r0; round < r1; ++round) {
        const uint32_t rk0 = k0 + (uint32_t)round * 0x9E3779B9u;
        const uint32_t rk1 = k1 + (uint32_t)round * 0xBB67AE85u;
        // one 32x32 -> 64-bit multiply each (v_mad_u64_u32) gives hi and lo
        const uint64_t p0 = (uint64_t)c.w[0] * 0xD2511F53u;
        const uint64_t p1 = (uint64_t)c.w[2] * 0xCD9E8D57u;
        // three-input XORs in one instruction each (truth table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c.w[1], rk0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c.w[3], rk1, 0x96);
        c.w[0] = n0;
        c.w[1] = (uint32_t)p1;
        c.w[2] = n2;
        c.w[3] = (uint32_t)p0;
    }
}

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1) {
    Words4 c{{c0, c1, c2, c3}};
    philox_rounds<0, 10>(c, k0, k1);
    return c;
}

// The Philox block that holds draw `slot` of (iteration, ant, step): counter
// ((slot >> 2) | (step << 16), ant, iteration, 0), key = the 64-bit seed.
// The draw is word (slot & 3) of the block.
__device__ __forceinline__ Words4 draw_block(uint64_t seed, uint32_t it, uint32_t ant, uint32_t step,
                                             uint32_t slot) {
    return philox4x32_10((slot >> 2) | (step << 16), ant, it, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ uint32_t pick_word(const Words4& b, uint32_t idx) {
    // idx in 0..3: a two-level select on its bits (the words stay in
    // registers; three selects and two bit tests)
    const bool lo = (idx & 1u) != 0u, hi = (idx & 2u) != 0u;
    const uint32_t w01 = lo ? b.w[1] : b.w[0];
    const uint32_t w23 = lo ? b.w[3] : b.w[2];
    return hi ? w23 : w01;
}

// u = (2 * (x >> 9) + 1) * 2^-24: exact, strictly inside (0, 1).
__device__ __forceinline__ float u01(uint32_t x) {
    return (float)(2u * (x >> 9) + 1u) * 0x1p-24f;
}

// Natural logarithm of u in (0, 1) in FP32 (every operation rounded on its
// own: the build disables contraction, and the fused multiply-adds are
// explicit). u = m 2^e with m in (sqrt(2)/2, sqrt(2)], f = m - 1 (exact),
// ln(1+f) = f + f^2 Q(f) where Q approximates (ln(1+f) - f) / f^2 by a
// degree-10 polynomial (a least-squares fit made for this project, weighted
// towards the minimax of f^2 |error|, coefficients rounded to FP32), by
// Horner's rule with v_fma_f32. ln 2 = kLn2Hi + kLn2Lo with a 15-bit head, so
// e kLn2Hi + f is exact for e in {-1, 0}; ln u = (e kLn2Hi + f) + (f^2 Q +
// e kLn2Lo). Within 0.83 ulp of ln u and monotone over all 2^23 draws.
__device__ __forceinline__ float log_u01(float u) {
    const float kLn2Hi = __uint_as_float(0x3F317200u);
    const float kLn2Lo = __uint_as_float(0x35BFBE8Eu);
    const float kSqrt2 = __uint_as_float(0x3FB504F3u);
    const uint32_t b = __float_as_uint(u);
    int e = (int)(b >> 23) - 127;
    float m = __uint_as_float((b & 0x007FFFFFu) | 0x3F800000u);
    if (m > kSqrt2) {
        m = m * 0.5f;
        e = e + 1;
    }
    const float f = m - 1.0f;
    float q = __uint_as_float(0xBD7C39FAu);               // f^10
    q = __builtin_fmaf(q, f, __uint_as_float(0x3DDE0BBCu));  // f^9
    q = __builtin_fmaf(q, f, __uint_as_float(0xBDDE3E43u));  // f^8
    q = __builtin_fmaf(q, f, __uint_as_float(0x3DE13229u));  // f^7
    q = __builtin_fmaf(q, f, __uint_as_float(0xBDFE32BFu));  // f^6
    q = __builtin_fmaf(q, f, __uint_as_float(0x3E124E2Fu));  // f^5
    q = __builtin_fmaf(q, f, __uint_as_float(0xBE2AB49Fu));  // f^4
    q = __builtin_fmaf(q, f, __uint_as_float(0x3E4CCCE5u));  // f^3
    q = __builtin_fmaf(q, f, __uint_as_float(0xBE7FFFD3u));  // f^2
    q = __builtin_fmaf(q, f, __uint_as_float(0x3EAAAAAAu));  // f
    q = __builtin_fmaf(q, f, -0.5f);                         // 1
    const float ef = (float)e;
    const float small = __builtin_fmaf(f * f, q, ef * kLn2Lo);
    return (ef * kLn2Hi + f) + small;
}

// x^k by left-to-right multiplication, x^0 = 1.
__device__ __forceinline__ float powi(float x, int k) {
    float r = 1.0f;
    for (int i = 0; i < k; ++i) r = r * x;
    return r;
}

// eta^beta with eta = 1/d.
__device__ __forceinline__ float heur_from_dist(int32_t d, int beta) {
    return powi(1.0f / (float)d, beta);
}

// Order-preserving map of a non-NaN float to uint32 (larger float -> larger
// code); every non-NaN float maps above 0, so 0 means "no key".
__device__ __forceinline__ uint32_t ord_key(float k) {
    const uint32_t b = __float_as_uint(k);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

// ---------------------------------------------------------------------------
// wave64 reductions. Rows of 16 lanes reduce through DPP lane permutations
// (quad swaps, half-row and row mirrors); the four row results are read into
// scalar registers and combined there. Every lane must be active.
// ---------------------------------------------------------------------------
template <int kCtrl>
__device__ __forceinline__ uint32_t dpp(uint32_t x) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, kCtrl, 0xF, 0xF, false);
}

// Inclusive prefix sum over the wave: row scans by DPP, row totals by readlane.
__device__ __forceinline__ int wave_incl_scan(int x, int lane) {
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
    const int r0 = __builtin_amdgcn_readlane(x, 15);
    const int r1 = __builtin_amdgcn_readlane(x, 31);
    const int r2 = __builtin_amdgcn_readlane(x, 47);
    const int row = lane >> 4;
    x += (row >= 1 ? r0 : 0) + (row >= 2 ? r1 : 0) + (row >= 3 ? r2 : 0);
    return x;
}

// kRows = number of 16-lane rows that hold data (2 for lanes 0..31, 4 for
// the whole wave).
template <int kRows = 4>
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    x = max(x, dpp<0xB1>(x));   // quad_perm [1,0,3,2]
    x = max(x, dpp<0x4E>(x));   // quad_perm [2,3,0,1]
    x = max(x, dpp<0x141>(x));  // row_half_mirror
    x = max(x, dpp<0x140>(x));  // row_mirror
    uint32_t r = max((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    if (kRows == 4)
        r = max(r, max((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48)));
    return r;
}

template <int kRows = 4>
__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    x = min(x, dpp<0xB1>(x));
    x = min(x, dpp<0x4E>(x));
    x = min(x, dpp<0x141>(x));
    x = min(x, dpp<0x140>(x));
    uint32_t r = min((uint32_t)__builtin_amdgcn_readlane((int)x, 0), (uint32_t)__builtin_amdgcn_readlane((int)x, 16));
    if (kRows == 4)
        r = min(r, min((uint32_t)__builtin_amdgcn_readlane((int)x, 32), (uint32_t)__builtin_amdgcn_readlane((int)x, 48)));
    return r;
}

__device__ __forceinline__ int64_t wave_sum_i64(int64_t x) {
    for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Argmax of (key code, -node) over the wave: the node with the largest key,
// the lowest node among equal keys. `code` is 0 for lanes without a key.
// Returns the node, or 0xFFFFFFFF if no lane had a key.
template <int kRows = 4>
__device__ __forceinline__ uint32_t wave_select(uint32_t code, uint32_t node) {
    const uint32_t best = wave_max_u32<kRows>(code);
    if (best == 0u) return 0xFFFFFFFFu;
    const uint64_t tied = __ballot(code == best);
    if (__popcll(tied) == 1) {
        const int lane = __ffsll((unsigned long long)tied) - 1;
        return (uint32_t)__builtin_amdgcn_readlane((int)node, lane);
    }
    return wave_min_u32<kRows>(code == best ? node : 0xFFFFFFFFu);
}

// The same selection, laid out for the construction step: the first holder
// of the best key is read before the (rare) test for a tie.
template <int kRows = 4>
__device__ __forceinline__ uint32_t wave_select_step(uint32_t code, uint32_t node) {
    const uint32_t best = wave_max_u32<kRows>(code);
    if (best == 0u) return 0xFFFFFFFFu;
    const uint64_t tied = __ballot(code == best);
    uint32_t sel = (uint32_t)__builtin_amdgcn_readlane((int)node, (int)__builtin_ctzll(tied));
    if (__builtin_expect((tied & (tied - 1)) != 0, 0)) sel = wave_min_u32<kRows>(code == best ? node : 0xFFFFFFFFu);
    return sel;
}

}  // namespace mmas

namespace mmas {

// Trail limits (Stuetzle and Hoos, with p_best): tau_max = 1/(rho C),
// tau_min = tau_max (1 - pdec) / ((n/2 - 1) pdec) with pdec = p_best^(1/n),
// in FP64 then rounded to FP32; tau_min never exceeds tau_max.
__device__ __forceinline__ void trail_limits(float rho, int64_t C, int n, double pdec, float* tmin,
                                             float* tmax) {
    const double hi = 1.0 / ((double)rho * (double)C);
    const double lo = (hi * (1.0 - pdec)) / (((double)n / 2.0 - 1.0) * pdec);
    const float fh = (float)hi;
    float fl = (float)lo;
    if (fl > fh) fl = fh;
    *tmin = fl;
    *tmax = fh;
}

// Lexicographic min of (value, index) packed as value << 32 | index for
// non-negative 31-bit values.
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    for (int o = 32; o >= 1; o >>= 1) {
        const uint64_t y = __shfl_xor(x, o);
        x = y < x ? y : x;
    }
    return x;
}

}  // namespace mmas
