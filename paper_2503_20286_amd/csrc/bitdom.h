// Block-bitset dominance (internal): candidate points are grouped in blocks of
// 64 (in sorted-position order).  For each block and objective the members'
// keys are kept sorted, with the bitmask of the first c members in that order
// for c = 0..64.  The members of a block that a point j dominates-or-ties in
// objective k are then one prefix mask, found by a 6-step binary search, and
// the members that dominate j are the AND of M such masks (restricted to
// positions before j's run).  One 64-bit mask replaces 64 * M compares.
#pragma once

#include "common.h"

namespace nsga3 {

constexpr int kBlk = 64;  // members per block

// Per-block table layout, in dwords:
//   [0..3]              header: min position, max position, member count, 0
//   [4..67]             member positions (ascending; padding 0x7fffffff)
//   [68 .. 68+64M)      per objective: the 64 member keys, sorted (padding 0xffffffff)
//   [68+64M .. +130M)   per objective: 65 prefix masks (entry c = first c members), as
//                       65 low dwords then 65 high dwords (a lane reading entry c hits
//                       bank c, so lanes with different counts do not conflict)
__host__ __device__ constexpr int blk_pos_off() { return 4; }
__host__ __device__ constexpr int blk_key_off(int k) { return 68 + 64 * k; }
__host__ __device__ constexpr int blk_pm_off(int M, int k) { return 68 + 64 * M + 130 * k; }
__host__ __device__ constexpr int blk_stride(int M) { return ((68 + 194 * M) + 3) / 4 * 4; }

// Number of the 64 sorted keys S that are <= x, in [0, 64] (S padded with
// 0xffffffff, and x is always below the padding).
__device__ __forceinline__ uint32_t count_le64(const uint32_t *S, uint32_t x) {
    uint32_t c = (S[31] <= x) ? 32u : 0u;
    c += (S[c + 15] <= x) ? 16u : 0u;
    c += (S[c + 7] <= x) ? 8u : 0u;
    c += (S[c + 3] <= x) ? 4u : 0u;
    c += (S[c + 1] <= x) ? 2u : 0u;
    c += (S[c] <= x) ? 1u : 0u;
    c += (c == 63u && S[63] <= x) ? 1u : 0u;  // six halvings reach 63 at most
    return c;
}

// Number of the 64 sorted keys S that are < x.
__device__ __forceinline__ uint32_t count_lt64(const uint32_t *S, uint32_t x) {
    uint32_t c = (S[31] < x) ? 32u : 0u;
    c += (S[c + 15] < x) ? 16u : 0u;
    c += (S[c + 7] < x) ? 8u : 0u;
    c += (S[c + 3] < x) ? 4u : 0u;
    c += (S[c + 1] < x) ? 2u : 0u;
    c += (S[c] < x) ? 1u : 0u;
    c += (c == 63u && S[63] < x) ? 1u : 0u;
    return c;
}

// Number of member positions (sorted, padded with 0x7fffffff) below bound.
__device__ __forceinline__ uint32_t count_pos_lt64(const int32_t *P, int32_t bound) {
    uint32_t c = (P[31] < bound) ? 32u : 0u;
    c += (P[c + 15] < bound) ? 16u : 0u;
    c += (P[c + 7] < bound) ? 8u : 0u;
    c += (P[c + 3] < bound) ? 4u : 0u;
    c += (P[c + 1] < bound) ? 2u : 0u;
    c += (P[c] < bound) ? 1u : 0u;
    c += (c == 63u && P[63] < bound) ? 1u : 0u;
    return c;
}

// Prefix mask entry c of objective table P (low dwords, then high dwords).
__device__ __forceinline__ uint64_t prefix_mask(const uint32_t *P, uint32_t c) {
    return (uint64_t)P[c] | ((uint64_t)P[65 + c] << 32);
}

// Lockstep form of count_le64 / count_lt64 for R independent searches (S[r]
// sorted 64-key arrays, x[r] the probes): every halving step issues all R
// reads before any compare, so the LDS latency is paid once per step.
// The search keeps a running pointer into S, so a step is one read (the
// step offset is an immediate), one compare, one select and one add.
template <int R, bool kLe>
__device__ __forceinline__ void count_many64(const uint32_t *const (&S)[R], const uint32_t (&x)[R],
                                             uint32_t (&c)[R]) {
    const uint32_t *p[R];
#pragma unroll
    for (int r = 0; r < R; ++r) p[r] = S[r] + ((kLe ? S[r][31] <= x[r] : S[r][31] < x[r]) ? 32 : 0);
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1) {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = p[r][step - 1];
#pragma unroll
        for (int r = 0; r < R; ++r) p[r] += (kLe ? v[r] <= x[r] : v[r] < x[r]) ? step : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        c[r] = (uint32_t)(p[r] - S[r]);
        c[r] += (c[r] == 63u && (kLe ? S[r][63] <= x[r] : S[r][63] < x[r])) ? 1u : 0u;
    }
}

__device__ __forceinline__ uint64_t low_bits(uint32_t c) {
    return c >= 64u ? ~0ull : ((1ull << c) - 1ull);
}

}  // namespace nsga3
