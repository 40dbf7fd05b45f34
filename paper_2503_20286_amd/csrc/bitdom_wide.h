// Wide block-bitset tables (internal): blocks of 128 sorted points instead of
// 64.  A probe of a wide block costs one more halving step and two more mask
// words per objective than a probe of a 64-member block but decides twice the
// pairs: at N = 200k, M = 5 the all-pairs counts issue 37 % fewer VALU
// instructions (495 M against 786 M per launch), and become bound by LDS
// instead (bank conflicts of the mask reads, five work-groups per CU).
// Dominance is as in bitdom.h (Listing 1 / Eq. (6) on order keys).
#pragma once

#include "bitdom.h"

namespace nsga3 {

constexpr int kWBlk = 128;  // members per wide block

// Wide table layout, in dwords:
//   [0..3]                   header: min position, max position, member count, 0
//   [4..131]                 member positions (ascending; padding 0x7fffffff)
//   [132 + 660k ..)          per objective k, four regions of 165 dwords (165 = 5 mod
//                            32, so that the keys a step of the search reads from
//                            different regions sit in different LDS banks): region r
//                            holds keys 32r..32r+31 (sorted; padding 0xffffffff), then
//                            four mask-word arrays of 33 entries.  Mask entry c (the set
//                            of the c members with the smallest keys) lives in region
//                            r = min(c / 32, 3) at entry c - 32r; its word q (members
//                            32q..32q+31) is 32 + 33q dwords after key slot c of r.
constexpr int kWRegion = 165;
__host__ __device__ constexpr int wblk_pos_off() { return 4; }
__host__ __device__ constexpr int wblk_obj_off(int k) { return 132 + 4 * kWRegion * k; }
__host__ __device__ constexpr int wblk_key_slot(int k, int c) {
    return wblk_obj_off(k) + kWRegion * (c >> 5) + (c & 31);
}
__host__ __device__ constexpr int wblk_mask(int k, int q, int c) {
    return wblk_obj_off(k) + kWRegion * (c < 128 ? c >> 5 : 3) + 32 + 33 * q +
           (c - 32 * (c < 128 ? c >> 5 : 3));
}
__host__ __device__ constexpr int wblk_stride(int M) { return (wblk_obj_off(M) + 3) / 4 * 4; }
static_assert(wblk_stride(4) == wide_blk_stride(4) && wblk_stride(10) == wide_blk_stride(10),
              "workspace sizing and the wide table layout disagree");

// Objective counts that count with wide tables: from M = 4 on the out-degrees
// come from the in-degree probes, and the probe is the cost; above M = 10 the
// wide probe's registers (251 VGPRs at M = 16) cost more occupancy than its
// instructions save (measured: M = 5 both counts 1.30 -> 1.25 ms, M = 10
// 0.58 -> 0.58 ms).
__host__ __device__ constexpr bool wide_counts(int M) { return M >= 4 && M <= 10; }

// Number of member positions (sorted, padded with 0x7fffffff) below bound.
__device__ __forceinline__ uint32_t count_pos_lt128(const int32_t *P, int32_t bound) {
    uint32_t c = (P[63] < bound) ? 64u : 0u;
    c += (P[c + 31] < bound) ? 32u : 0u;
    c += (P[c + 15] < bound) ? 16u : 0u;
    c += (P[c + 7] < bound) ? 8u : 0u;
    c += (P[c + 3] < bound) ? 4u : 0u;
    c += (P[c + 1] < bound) ? 2u : 0u;
    c += (P[c] < bound) ? 1u : 0u;
    c += (c == 127u && P[127] < bound) ? 1u : 0u;
    return c;
}

// Wide table b of a list of n records (MP-dword records: M keys, then the
// sorted position), objective k0, k0 + kstep, ... by this wave; objective 0
// also writes the header and positions.  Lane l holds members l and l + 64.
template <int M>
__device__ __forceinline__ void build_wide_at(const uint32_t *__restrict__ rec, int32_t n,
                                              uint32_t *T, int32_t b, int32_t *inv, int k0,
                                              int kstep) {
    constexpr int MP = rec_stride(M);
    if ((int64_t)b * kWBlk >= n) return;
    const int l = (int)lane_id();
    const int32_t e0 = b * kWBlk + l, e1 = e0 + kWave;
    const bool v0 = e0 < n, v1 = e1 < n;
    const int32_t nmem = min(kWBlk, n - b * kWBlk);
    if (k0 == 0) {
        const int32_t p0 = v0 ? (int32_t)rec[(size_t)e0 * MP + M] : 0x7fffffff;
        const int32_t p1 = v1 ? (int32_t)rec[(size_t)e1 * MP + M] : 0x7fffffff;
        T[wblk_pos_off() + l] = (uint32_t)p0;
        T[wblk_pos_off() + kWave + l] = (uint32_t)p1;
        const int32_t li = nmem - 1;
        const int32_t last = li < kWave ? __shfl(p0, li, 64) : __shfl(p1, li - kWave, 64);
        const int32_t first = __shfl(p0, 0, 64);
        if (l == 0) {
            T[0] = (uint32_t)first;
            T[1] = (uint32_t)last;
            T[2] = (uint32_t)nmem;
            T[3] = 0;
        }
    }
    for (int k = k0; k < M; k += kstep) {
        const uint32_t x0 = v0 ? rec[(size_t)e0 * MP + k] : 0xffffffffu;
        const uint32_t x1 = v1 ? rec[(size_t)e1 * MP + k] : 0xffffffffu;
        // rank among the 128 keys, ties by member index (member m of lane s is
        // s, member m + 64 is s + 64)
        uint32_t r0 = 0, r1 = 0;
#pragma unroll 16
        for (int s = 0; s < kWave; ++s) {
            const uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)x0, s);
            const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)x1, s);
            r0 += (a < x0 || (a == x0 && s < l)) ? 1u : 0u;
            r0 += (c < x0) ? 1u : 0u;  // member s + 64 > member l
            r1 += (a <= x1) ? 1u : 0u;  // member s < member l + 64
            r1 += (c < x1 || (c == x1 && s < l)) ? 1u : 0u;
        }
        T[wblk_key_slot(k, (int)r0)] = x0;
        T[wblk_key_slot(k, (int)r1)] = x1;
        inv[r0] = l;
        inv[r1] = l + kWave;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // prefix masks: entry c + 1 holds the members of ranks 0..c
        const int m0 = inv[l], m1 = inv[kWave + l];
        uint32_t lo[4], hi[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const uint32_t b0 = (m0 < nmem && (m0 >> 5) == q) ? (1u << (m0 & 31)) : 0u;
            const uint32_t b1 = (m1 < nmem && (m1 >> 5) == q) ? (1u << (m1 & 31)) : 0u;
            lo[q] = wave_inclusive_scan<true>(b0);
            hi[q] = wave_inclusive_scan<true>(b1) |
                    (uint32_t)__builtin_amdgcn_readlane((int)lo[q], kWave - 1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            T[wblk_mask(k, q, l + 1)] = lo[q];
            T[wblk_mask(k, q, kWave + l + 1)] = hi[q];
            if (l == 0) T[wblk_mask(k, q, 0)] = 0u;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// For R probes of wide table T: the prefix mask (four words) of objective k[r]
// at "number of member keys <= x[r]".  Two steps pick the region (keys 63,
// then 32r + 31), five halving steps and a last one-key step follow inside it,
// each one read, one compare, one select and one add; all R reads of a step
// are issued before any compare.  A search ends on key slot c of its region,
// and mask entry c lies at fixed distances from it.
template <int M, int R>
__device__ __forceinline__ void masks_many128(const uint32_t *T, const int (&k)[R],
                                              const uint32_t (&x)[R], uint32_t (&mask)[R][4]) {
    const uint32_t base = lds_addr(T);
    uint32_t a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t o = base + 4u * (uint32_t)wblk_obj_off(k[r]);
        const uint32_t v = lds_ld(o + 4u * (uint32_t)(kWRegion + 31));  // key 63
        a[r] = o + ((v <= x[r]) ? 4u * 2u * kWRegion : 0u);
    }
    {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_ld(a[r] + 4u * 31u);  // key 32r + 31
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] += (v[r] <= x[r]) ? 4u * kWRegion : 0u;
    }
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1) {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_ld(a[r] + 4u * (uint32_t)(step - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] += (v[r] <= x[r]) ? 4u * step : 0u;
    }
    {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_ld(a[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] += (v[r] <= x[r]) ? 4u : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) mask[r][q] = lds_ld(a[r] + 4u * (uint32_t)(32 + 33 * q));
}

__device__ __forceinline__ void low_bits128(uint32_t c, uint32_t (&m)[4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t lo = 32u * (uint32_t)q;
        m[q] = c >= lo + 32u ? ~0u : (c <= lo ? 0u : ((1u << (c - lo)) - 1u));
    }
}

// fwd_blocks over nb staged wide tables: each lane's TJ points j gain the
// number of members that dominate them (members before j's run); with kOut
// every dominating member gains one in its LDS counter oc[b * 128 + member].
template <int M, int TJ, bool kOut>
__device__ __forceinline__ void fwd_blocks_wide(const uint32_t *lt, int32_t nb, int32_t run_lo,
                                                int32_t run_hi, const uint32_t (&kj)[TJ][M],
                                                const int32_t (&run)[TJ], int32_t (&cnt)[TJ],
                                                uint32_t *oc) {
    constexpr int TS = wblk_stride(M);
    for (int32_t b = 0; b < nb; ++b) {
        const uint32_t *T = lt + b * TS;
        const int32_t bmin = (int32_t)T[0];
        const int32_t bmax = (int32_t)T[1];
        if (bmin >= run_hi) break;  // later blocks start later still
        const bool full = bmax < run_lo;
        int ko[TJ * M];
        uint32_t x[TJ * M];
        uint32_t pm[TJ * M][4];
#pragma unroll
        for (int t = 0; t < TJ; ++t)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                ko[t * M + k] = k;
                x[t * M + k] = kj[t][k];
            }
        masks_many128<M, TJ * M>(T, ko, x, pm);
        uint32_t mt[TJ][4];
#pragma unroll
        for (int t = 0; t < TJ; ++t) {
            uint32_t m[4] = {~0u, ~0u, ~0u, ~0u};
            if (!full) {
                if (run[t] <= bmin) {
                    m[0] = m[1] = m[2] = m[3] = 0u;
                } else if (run[t] <= bmax) {
                    low_bits128(count_pos_lt128(reinterpret_cast<const int32_t *>(T + wblk_pos_off()),
                                                run[t]), m);
                }
            }
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int q = 0; q < 4; ++q) m[q] &= pm[t * M + k][q];
            cnt[t] += __popc(m[0]) + __popc(m[1]) + __popc(m[2]) + __popc(m[3]);
#pragma unroll
            for (int q = 0; q < 4; ++q) mt[t][q] = m[q];
        }
        if constexpr (kOut) {
            uint32_t *ob = oc + b * kWBlk;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                uint32_t u = 0u;
#pragma unroll
                for (int t = 0; t < TJ; ++t) u |= mt[t][q];
                while (u) {
                    const uint32_t bit = (uint32_t)__builtin_ctz(u);
                    uint32_t n = 0;
#pragma unroll
                    for (int t = 0; t < TJ; ++t) n += (mt[t][q] >> bit) & 1u;
                    __hip_atomic_fetch_add(ob + 32 * q + bit, n, __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_WORKGROUP);
                    u &= u - 1u;
                }
            }
        }
    }
}

// Stage nb consecutive wide tables into LDS.
template <int M>
__device__ __forceinline__ void stage_wide(uint32_t *lds, const uint32_t *__restrict__ tabs,
                                           int32_t b0, int32_t nb) {
    constexpr int TS = wblk_stride(M);
    const uint4 *src = reinterpret_cast<const uint4 *>(tabs + (size_t)b0 * TS);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    for (int q = threadIdx.x; q < nb * (TS / 4); q += kFwdThreads) dst[q] = src[q];
}

// fwd_level_group with wide tables of the front: one tile of kFwdThreads * TJ
// remaining points (keys in registers) against ng consecutive chunks of cb
// wide tables from table b0 on, one atomic per point.
template <int M, int TJ>
__device__ __forceinline__ void fwd_level_group_wide(const uint32_t *__restrict__ tabs,
                                                     int32_t b0, int32_t cb, int32_t ng,
                                                     int32_t nblk, const uint32_t *__restrict__ uk,
                                                     const int32_t *__restrict__ urun, int32_t nu,
                                                     int32_t *__restrict__ ucnt, int32_t jt,
                                                     uint32_t *lt) {
    constexpr int TS = wblk_stride(M);
    constexpr int TILE = kFwdThreads * TJ;
    if (jt * TILE >= nu) return;
    const int32_t last_run = vld(&urun[min((jt + 1) * TILE, nu) - 1]);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    const int32_t jbase = jt * TILE + w * kWave * TJ;
    const bool active = jbase < nu;  // uniform in the wave
    uint32_t kj[TJ][M];
    int32_t run[TJ], cnt[TJ];
    int32_t run_lo = 0, run_hi = 0;
#pragma unroll
    for (int u = 0; u < TJ; ++u) cnt[u] = 0;
    if (active) {
        load_points<M, TJ>(uk, urun, nu, jbase, lane, kj, run);
        run_lo = vld(&urun[jbase]);
        run_hi = vld(&urun[min(jbase + kWave * TJ - 1, nu - 1)]);
    }
    for (int32_t g = 0; g < ng; ++g) {
        const int32_t bs = b0 + g * cb;
        if (bs >= nblk) break;
        if ((int32_t)vld(&tabs[(size_t)bs * TS]) >= last_run) break;
        const int32_t nb = min(cb, nblk - bs);
        __syncthreads();  // every wave is done with the previous chunk
        stage_wide<M>(lt, tabs, bs, nb);
        __syncthreads();
        if (active) fwd_blocks_wide<M, TJ, false>(lt, nb, run_lo, run_hi, kj, run, cnt, nullptr);
    }
    if (active) {
#pragma unroll
        for (int u = 0; u < TJ; ++u) {
            const int32_t q = jbase + u * kWave + lane;
            if (q < nu && cnt[u]) atomicSub(&ucnt[q], cnt[u]);
        }
    }
}

}  // namespace nsga3
