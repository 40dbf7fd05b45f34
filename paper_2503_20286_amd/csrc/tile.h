// Pairwise dominance tile core shared by the dominance-count and peeling
// kernels of libnsga3 (internal).
#pragma once

#include "common.h"
#include "prims.h"

namespace nsga3 {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kT = 4;                     // j points per lane
constexpr int kJT = kThreads * kT;        // j points per tile (block)
constexpr int kIC = kJT;                  // i points per chunk (dominance count)

// ---------------------------------------------------------------------------
// Pairwise tile core.  The calling wave holds kT * 64 "later" points in
// registers (keys kj, run starts run); the "earlier" points stream through
// scalar registers from a record array.  For each earlier point the M compares
// produce 64-bit lane masks that are combined on the scalar unit; the lane
// count of the later point is bumped from the mask, and the popcount of the
// mask is the number of later points the earlier one dominates.
// ---------------------------------------------------------------------------
// cnt += bit `lane` of mask, as one VALU op (add with the mask as carry-in).
__device__ __forceinline__ void add_mask_bit(int32_t &cnt, uint64_t mask) {
    uint64_t carry_out;
    asm volatile("v_addc_co_u32_e64 %0, %1, 0, %0, %2" : "+v"(cnt), "=s"(carry_out) : "s"(mask));
}

// Dominance masks of one earlier point (keys ki, sorted position ipos) over
// the wave's kT * 64 later points.  Bumps cin and returns the total count.
template <int M, bool kChecked, bool kCountOut>
__device__ __forceinline__ uint32_t tile_one(const uint32_t (&ki)[M], int ipos,
                                             const uint32_t (&kj)[kT][M],
                                             const int32_t (&run)[kT], int32_t (&cin)[kT]) {
    uint32_t c = 0;
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        uint64_t m = ballot(ki[0] <= kj[t][0]);
#pragma unroll
        for (int k = 1; k < M; ++k) m &= ballot(ki[k] <= kj[t][k]);
        if (kChecked) m &= ballot(ipos < run[t]);
        add_mask_bit(cin[t], m);
        if (kCountOut) c += (uint32_t)__popcll(m);
    }
    return c;
}

// Streams n earlier records (sorted by position) against the wave's later
// points.  Records are fetched in groups of kU so the scalar loads overlap;
// RecPtr is a global pointer (scalar loads), a constant-address-space
// pointer (scalar loads forced) or an LDS pointer.
// With kCountOut, lane 0 stores the per-record counts to out_row[0..n).
template <int M, bool kChecked, bool kCountOut, typename RecPtr>
__device__ __forceinline__ void tile_rows(RecPtr __restrict__ rec, int n,
                                          const uint32_t (&kj)[kT][M], const int32_t (&run)[kT],
                                          int32_t (&cin)[kT], uint32_t *__restrict__ out_row,
                                          bool lane0) {
    constexpr int kU = 4;
    constexpr int MP = rec_stride(M);
    int ii = 0;
    for (; ii + kU <= n; ii += kU) {
        uint32_t ki[kU][M];
        int ipos[kU];
        const RecPtr g = rec + (size_t)ii * MP;  // one base, constant offsets
#pragma unroll
        for (int u = 0; u < kU; ++u) {
#pragma unroll
            for (int k = 0; k < M; ++k) ki[u][k] = g[u * MP + k];
            ipos[u] = kChecked ? (int)g[u * MP + M] : 0;
        }
        uint32_t c[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            c[u] = tile_one<M, kChecked, kCountOut>(ki[u], ipos[u], kj, run, cin);
            // keep the masks of one record live at a time (no SGPR spills)
            __builtin_amdgcn_sched_barrier(0);
        }
        if (kCountOut && lane0) {
#pragma unroll
            for (int u = 0; u < kU; ++u) out_row[ii + u] = c[u];
        }
    }
    for (; ii < n; ++ii) {
        const RecPtr r = rec + (size_t)ii * MP;
        uint32_t ki[M];
#pragma unroll
        for (int k = 0; k < M; ++k) ki[k] = r[k];
        const int ipos = kChecked ? (int)r[M] : 0;
        const uint32_t c = tile_one<M, kChecked, kCountOut>(ki, ipos, kj, run, cin);
        if (kCountOut && lane0) out_row[ii] = c;
    }
}


// Like tile_rows (no per-record counts), for a position-sorted record list
// that may extend past the wave's points: stops at the first record whose
// position is >= run_hi, and skips the run-start check for groups that lie
// entirely before run_lo.
template <int M>
__device__ __forceinline__ void tile_rows_bounded(const uint32_t *__restrict__ rec, int n,
                                                  int run_lo, int run_hi,
                                                  const uint32_t (&kj)[kT][M],
                                                  const int32_t (&run)[kT], int32_t (&cin)[kT]) {
    constexpr int kU = 4;
    constexpr int MP = rec_stride(M);
    int ii = 0;
    for (; ii + kU <= n; ii += kU) {
        uint32_t ki[kU][M];
        int ipos[kU];
        const uint32_t *g = rec + (size_t)ii * MP;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
#pragma unroll
            for (int k = 0; k < M; ++k) ki[u][k] = g[u * MP + k];
            ipos[u] = (int)g[u * MP + M];
        }
        if (ipos[0] >= run_hi) return;
        if (ipos[kU - 1] < run_lo) {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                tile_one<M, false, false>(ki[u], ipos[u], kj, run, cin);
                __builtin_amdgcn_sched_barrier(0);
            }
        } else {
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                tile_one<M, true, false>(ki[u], ipos[u], kj, run, cin);
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    }
    for (; ii < n; ++ii) {
        const uint32_t *r = rec + (size_t)ii * MP;
        uint32_t ki[M];
#pragma unroll
        for (int k = 0; k < M; ++k) ki[k] = r[k];
        const int ipos = (int)r[M];
        if (ipos >= run_hi) return;
        tile_one<M, true, false>(ki, ipos, kj, run, cin);
    }
}

}  // namespace nsga3
