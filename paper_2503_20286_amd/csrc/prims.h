// Device primitives for libnsga3: wave helpers, a stable LSD radix sort of
// (uint64 key, uint32 value) pairs, ordered stream compaction, and a grid
// barrier for cooperative launches.
#pragma once

#include "common.h"

namespace nsga3 {

__device__ __forceinline__ uint32_t lane_id() {
    return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
}

// Number of set bits of `mask` in lanes below the calling lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_min(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w < v ? w : v;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
    for (int o = 32; o > 0; o >>= 1) {
        T w = __shfl_xor(v, o, 64);
        v = w > v ? w : v;
    }
    return v;
}

// Inclusive scan (OR or sum) over a wave's 64 lanes with data-parallel
// primitive moves instead of LDS permutes: shifts by 1, 2, 4 and 8 lanes
// within each row of 16, then lane 15 broadcast into rows 1 and 3 and lane 31
// into rows 2 and 3.  A lane whose source lies outside its row (or whose row
// a broadcast skips) reads 0, the identity of both operations.  Every lane of
// the wave must be active.
template <bool kOr>
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t x) {
#define NSGA3_DPP_STEP(ctrl, rows)                                                          \
    {                                                                                       \
        const uint32_t t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, ctrl, rows, 0xf, \
                                                                 false);                    \
        x = kOr ? (x | t) : (x + t);                                                        \
    }
    NSGA3_DPP_STEP(0x111, 0xf)  // row_shr:1
    NSGA3_DPP_STEP(0x112, 0xf)  // row_shr:2
    NSGA3_DPP_STEP(0x114, 0xf)  // row_shr:4
    NSGA3_DPP_STEP(0x118, 0xf)  // row_shr:8
    NSGA3_DPP_STEP(0x142, 0xa)  // row_bcast:15
    NSGA3_DPP_STEP(0x143, 0xc)  // row_bcast:31
#undef NSGA3_DPP_STEP
    return x;
}

// Block-wide exclusive scan of one uint32 per thread (blockDim.x a multiple of
// 64, at most 1024).  Returns the exclusive prefix; *total receives the sum.
// `lds` needs blockDim.x / 64 + 1 entries.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t *total) {
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    const uint32_t incl = wave_inclusive_scan<false>(v);
    if (lane == kWave - 1) lds[wid] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t w = 0; w < nw; ++w) {
            uint32_t t = lds[w];
            lds[w] = run;
            run += t;
        }
        lds[nw] = run;
    }
    __syncthreads();
    uint32_t res = lds[wid] + incl - v;
    *total = lds[nw];
    __syncthreads();
    return res;
}

// ---------------------------------------------------------------------------
// Grid barriers for cooperative (co-resident) launches.  Every block of the
// grid must call them the same number of times.  Memory ordering: each block's
// thread 0 issues one release fence before arriving (its block's writes become
// visible device-wide) and one acquire fence after leaving; arrival counters
// and release flags use relaxed device-scope atomics, and polling uses relaxed
// loads so that it does not invalidate caches on every probe.  A bounded spin
// turns a lost block into an error flag instead of a hang; blocks then leave
// their loops.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool barrier_spin(const uint32_t *flag, uint32_t g, uint32_t *err) {
    uint64_t spins = 0;
    while (__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
        __builtin_amdgcn_s_sleep(2);
        ++spins;
        if ((spins & 1023u) == 0 &&
            (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrBarrierTimeout))
            return false;
        if (spins > (1ull << 26)) {  // far beyond any legitimate wait
            __hip_atomic_fetch_or(err, (uint32_t)kErrBarrierTimeout, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
    }
    return true;
}

// Flat form: one arrival counter and one generation word.
__device__ __forceinline__ bool grid_barrier(uint32_t *count, uint32_t *gen, uint32_t *err,
                                             uint32_t nblocks) {
    __syncthreads();
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) {
        bool ok = true;
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // publish this block's writes
        const uint32_t arrived =
            __hip_atomic_fetch_add(count, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(gen, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            ok = barrier_spin(gen, g, err);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // see every block's writes
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrBarrierTimeout)
            ok = false;
        s_ok = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok != 0;
}

// Two-level form (see GridBar): arrivals spread over kBarSub counters.
__device__ __forceinline__ bool grid_barrier2(GridBar *bar, uint32_t *err) {
    __syncthreads();
    __shared__ uint32_t s_ok2;
    if (threadIdx.x == 0) {
        bool ok = true;
        const uint32_t G = gridDim.x;
        const uint32_t nsub = G < (uint32_t)kBarSub ? G : (uint32_t)kBarSub;
        const uint32_t sub = blockIdx.x % nsub;
        const uint32_t members = G / nsub + (sub < G % nsub ? 1u : 0u);
        uint32_t *flag = &bar->flag[sub].v;
        const uint32_t g = __hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        bool released = false;
        const uint32_t a = __hip_atomic_fetch_add(&bar->count[sub].v, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (a == members - 1) {
            __hip_atomic_store(&bar->count[sub].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
            const uint32_t r = __hip_atomic_fetch_add(&bar->root.v, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            if (r == nsub - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                __hip_atomic_store(&bar->root.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
                for (uint32_t q = 0; q < nsub; ++q)
                    __hip_atomic_store(&bar->flag[q].v, g + 1u, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) ok = barrier_spin(flag, g, err);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrBarrierTimeout)
            ok = false;
        s_ok2 = ok ? 1u : 0u;
    }
    __syncthreads();
    return s_ok2 != 0;
}

}  // namespace nsga3
