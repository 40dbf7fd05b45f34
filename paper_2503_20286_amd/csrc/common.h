// Internal definitions shared by the kernels and the host runtime of libnsga3.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nsga3.h"

namespace nsga3 {

constexpr int kWave = 64;

// Record stride (dwords) of one point in the sorted array-of-structures used by
// the pairwise kernels: M order keys followed by the point's sorted position,
// padded to a power of two so that one scalar load fetches a whole record.
__host__ __device__ constexpr int rec_stride(int M) {
    return (M + 1) <= 4 ? 4 : (M + 1) <= 8 ? 8 : (M + 1) <= 16 ? 16 : 32;
}

// Order-preserving map float32 -> uint32: a < b (IEEE) <=> key(a) < key(b) for
// finite values; -0 and +0 map to the same key.
__device__ __forceinline__ uint32_t order_key(float f) {
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7fffffffu) == 0u) b = 0u;
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float key_to_float(uint32_t k) {
    uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
    return __uint_as_float(b);
}

// Device-side status flags (bit set => error found on device).
enum : uint32_t {
    kErrNonfiniteObj = 1u,
    kErrBadRef = 2u,
    kErrInternal = 4u,
    kErrBarrierTimeout = 8u,
};

// Peeling levels whose sizes go back to the host after each call.
constexpr int kProfLevels = 64;

// Small per-call scalars kept in device memory.
struct DevScalars {
    uint32_t err;              // kErr* bits
    uint32_t min_key[16];      // per-objective minimum order key (ideal point)
    int32_t last_front;        // l
    int32_t num_fronts;        // L
    int32_t last_front_size;   // |F_l|
    int64_t n_before;          // #{rank < l}
    int64_t num_from_last;     // R
    int32_t fallback;          // intercept fallback code
    int32_t near_ties;
    int32_t nf, nu;            // peeling list sizes (current level)
    uint32_t bar_count;        // grid barrier (flat form)
    uint32_t bar_gen;
    int32_t level_V;           // niching threshold level
    int32_t ref_thr;           // niching threshold reference
    uint32_t n_selected;       // number of selection flags set (must equal K)
    double a[16];              // intercepts
    double z[16];              // ideal point (float64 of the float32 minimum)
    int32_t fb[1 + kProfLevels];  // front count, then points left after each level
};

// Two-level grid barrier state: blocks arrive on one of kBarSub counters
// (each on its own 128-byte line), the last arriver of a group arrives at the
// root, and the last group releases every group's flag.  Keeping arrivals and
// polling spread over separate lines avoids one hot address.
constexpr int kBarSub = 16;
struct alignas(128) BarLine {
    uint32_t v;
    uint32_t pad[31];
};
struct GridBar {
    BarLine count[kBarSub];
    BarLine flag[kBarSub];
    BarLine root;
};

struct Ws;  // workspace views, defined in the runtime

// Dwords of one 64-member block-bitset table of an M-objective point list
// (header and positions, then 195 dwords per objective: keys and prefix
// masks, laid out in bitdom.h), rounded to whole 16-byte vectors.
__host__ __device__ constexpr int blk_stride(int M) { return ((68 + 195 * M) + 3) / 4 * 4; }

// Dwords of one 128-member (wide) table (header and positions, then 660 dwords
// per objective, laid out in bitdom_wide.h), rounded to whole 16-byte vectors.
__host__ __device__ constexpr int wide_blk_stride(int M) { return ((132 + 660 * M) + 3) / 4 * 4; }

}  // namespace nsga3
