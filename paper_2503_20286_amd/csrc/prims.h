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

// Block-wide exclusive scan of one uint32 per thread (blockDim.x a multiple of
// 64, at most 1024).  Returns the exclusive prefix; *total receives the sum.
// `lds` needs blockDim.x / 64 + 1 entries.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds, uint32_t *total) {
    const uint32_t lane = lane_id();
    const uint32_t wid = threadIdx.x / kWave;
    const uint32_t nw = blockDim.x / kWave;
    uint32_t incl = v;
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= (uint32_t)o) incl += t;
    }
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
// Grid barrier for cooperative (co-resident) launches.  Every block of the grid
// must call it the same number of times.  A bounded spin turns a lost block
// into an error flag instead of a hang; blocks then leave their loops.
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool grid_barrier(uint32_t *count, uint32_t *gen, uint32_t *err,
                                             uint32_t nblocks) {
    __syncthreads();
    __shared__ uint32_t s_ok;
    if (threadIdx.x == 0) {
        uint32_t ok = 1;
        const uint32_t g = __hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        __threadfence();
        const uint32_t arrived =
            __hip_atomic_fetch_add(count, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_add(gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint64_t spins = 0;
            while (__hip_atomic_load(gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == g) {
                __builtin_amdgcn_s_sleep(2);
                ++spins;
                if ((spins & 1023u) == 0 &&
                    (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                     kErrBarrierTimeout)) {
                    ok = 0;
                    break;
                }
                if (spins > (1ull << 26)) {  // far beyond any legitimate wait
                    __hip_atomic_fetch_or(err, (uint32_t)kErrBarrierTimeout, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
            }
        }
        __threadfence();
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrBarrierTimeout)
            ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

}  // namespace nsga3
