// Block-bitset dominance (internal): candidate points are grouped in blocks of
// 64 (in sorted-position order).  For each block and objective the members'
// keys are kept sorted, with the bitmask of the first c members in that order
// for c = 0..64.  The members of a block that a point j dominates-or-ties in
// objective k are then one prefix mask, found by a 6-step binary search, and
// the members that dominate j are the AND of M such masks (restricted to
// positions before j's run).  One 64-bit mask replaces 64 * M compares.
#pragma once

#include "common.h"
#include "prims.h"

namespace nsga3 {

constexpr int kBlk = 64;  // members per block

// Per-block table layout, in dwords:
//   [0..3]              header: min position, max position, member count, 0
//   [4..67]             member positions (ascending; padding 0x7fffffff)
//   [68 + 195k ..)      per objective k, two regions 97 dwords apart (97 = 1 mod 32:
//                       one LDS bank apart), for the member-key ranks c < 32 and c >= 32:
//                         lower  [keys 0..31 | mask lows c = 0..31 | 1 spare | mask highs 0..31]
//                         upper  [keys 32..63 | mask lows c = 32..64 | mask highs 32..64]
//                       keys sorted (padding 0xffffffff); mask entry c is the set of the c
//                       members with the smallest keys, its low dword 32 and its high dword
//                       65 dwords after key slot c (key slot 64 being one past key 63)
__host__ __device__ constexpr int blk_pos_off() { return 4; }
constexpr int kBlkUpper = 97;   // upper region offset in dwords
__host__ __device__ constexpr int blk_obj_off(int k) { return 68 + 195 * k; }
__host__ __device__ constexpr int blk_key_slot(int k, int c) {
    return c < 32 ? blk_obj_off(k) + c : blk_obj_off(k) + kBlkUpper + (c - 32);
}
__host__ __device__ constexpr int blk_mask_lo(int k, int c) { return blk_key_slot(k, c) + 32; }
__host__ __device__ constexpr int blk_mask_hi(int k, int c) { return blk_key_slot(k, c) + 65; }
// (blk_stride(M), the table size in dwords, is in common.h: the batched
// engine's workspace layout needs it too.)
static_assert(blk_stride(16) >= blk_obj_off(16), "table stride covers every objective");

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

// LDS byte addresses.  A generic pointer to LDS holds the LDS offset in its
// low 32 bits, so the searches below work on 32-bit LDS addresses.
typedef __attribute__((address_space(3))) const uint32_t lds_cu32;
__device__ __forceinline__ uint32_t lds_addr(const uint32_t *p) { return (uint32_t)(uintptr_t)p; }
__device__ __forceinline__ uint32_t lds_ld(uint32_t a) { return *(lds_cu32 *)(uintptr_t)a; }

// For R independent probes of block table T: the prefix mask of objective
// k[r] at "number of member keys <= x[r]" (kLe) or "< x[r]".  Each search
// keeps a running LDS address: the first step picks the lower or the upper
// region (32 keys each), five halving steps and a last one-key step follow
// inside that region, each one read (the step is the instruction's immediate
// offset), one compare, one select and one add; all R reads of a step are
// issued before any compare.  The regions sit one bank apart, so lanes that
// search the same block in different halves do not conflict.  The search ends
// on key slot c, and mask entry c lies at fixed distances from it.
template <int M, int R, bool kLe>
__device__ __forceinline__ void masks_many64(const uint32_t *T, const int (&k)[R],
                                             const uint32_t (&x)[R], uint64_t (&mask)[R]) {
    const uint32_t base = lds_addr(T);
    uint32_t a[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t lo = base + 4u * (uint32_t)blk_obj_off(k[r]);
        const uint32_t v = lds_ld(lo + 4u * 31u);
        a[r] = lo + ((kLe ? v <= x[r] : v < x[r]) ? 4u * kBlkUpper : 0u);
    }
#pragma unroll
    for (int step = 16; step >= 1; step >>= 1) {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_ld(a[r] + 4u * (uint32_t)(step - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] += (kLe ? v[r] <= x[r] : v[r] < x[r]) ? 4u * step : 0u;
    }
    {
        uint32_t v[R];
#pragma unroll
        for (int r = 0; r < R; ++r) v[r] = lds_ld(a[r]);
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] += (kLe ? v[r] <= x[r] : v[r] < x[r]) ? 4u : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t lo = lds_ld(a[r] + 4u * 32u);
        const uint32_t hi = lds_ld(a[r] + 4u * 65u);
        mask[r] = (uint64_t)lo | ((uint64_t)hi << 32);
    }
}

__device__ __forceinline__ uint64_t low_bits(uint32_t c) {
    return c >= 64u ? ~0ull : ((1ull << c) - 1ull);
}

// ---------------------------------------------------------------------------
// Device bodies shared by the single-selection kernels (bitdom.hip) and the
// batched engine (engine.hip).
// ---------------------------------------------------------------------------
constexpr int kFwdThreads = 256;
constexpr int kTJ = 2;                            // points per lane
constexpr int kTileJ = kFwdThreads * kTJ;         // points per work item
// Tables staged per work-group: the 64-member all-pairs counts take 24.5 KiB
// chunks (six M = 5 tables; with the out-degree counters six work-groups stay
// resident per CU: 2.98 ms for both counts at N = 200k, M = 5 when they were
// separate passes, against 3.24 ms with 34 KiB and 3.81 ms with 49 KiB); the
// batched engine's peeling items take 34 KiB (kLdsLevelDwords), the single
// call's level kernel 24 KiB (kLdsLevelKernelDwords, below).
#ifndef NSGA3_LDS_COUNT_DWORDS
#define NSGA3_LDS_COUNT_DWORDS 6264
#endif
constexpr int kLdsCountDwords = NSGA3_LDS_COUNT_DWORDS;
constexpr int kLdsLevelDwords = 8704;

template <int Dwords, int M>
__host__ __device__ constexpr int chunk_blocks() {
    return Dwords / blk_stride(M) < 1 ? 1 : Dwords / blk_stride(M);
}
template <int M>
__host__ __device__ constexpr int count_chunk() { return chunk_blocks<kLdsCountDwords, M>(); }
template <int M>
__host__ __device__ constexpr int level_chunk() { return chunk_blocks<kLdsLevelDwords, M>(); }
// The single-call level kernel stages smaller chunks than the engine's items:
// 24 KiB lets six of its work-groups stay resident per CU (peel at N = 200k,
// M = 5: 1.090 ms with 24 KiB and six per CU, 1.112 with 34 KiB and four).
constexpr int kLdsLevelKernelDwords = 6264;
template <int M>
__host__ __device__ constexpr int level_kernel_chunk() { return chunk_blocks<kLdsLevelKernelDwords, M>(); }

// ---------------------------------------------------------------------------
// Tables: one wave per block of 64 consecutive list entries.
// ---------------------------------------------------------------------------
template <bool kWaveSync>
__device__ __forceinline__ void block_sync() {
    if constexpr (kWaveSync) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// kWaveSync: the calling wave builds its block alone (work-groups of several
// waves, each with its own inv[64]); otherwise the work-group is this one wave.
// The calling wave writes the objectives k0, k0 + kstep, ... of the table
// (and the header and positions when k0 == 0), so several waves can share one
// table.
template <int M, bool kWaveSync = false>
__device__ __forceinline__ void build_block_at(const uint32_t *__restrict__ rec, int32_t n,
                                               uint32_t *T, int32_t b, int32_t *inv, int k0,
                                               int kstep) {
    constexpr int MP = rec_stride(M);
    if ((int64_t)b * kBlk >= n) return;
    const int l = (int)lane_id();
    const int32_t e = b * kBlk + l;
    const bool valid = e < n;
    const int32_t nmem = min(kBlk, n - b * kBlk);
    if (k0 == 0) {
        const int32_t pos = valid ? (int32_t)rec[(size_t)e * MP + M] : 0x7fffffff;
        T[blk_pos_off() + l] = (uint32_t)pos;
        // (no uniform-address loads: a persistent caller's records change
        // between stages, and a scalar load could hit a stale scalar-cache line)
        const int32_t last = __shfl(pos, nmem - 1, 64);
        if (l == 0) {
            T[0] = (uint32_t)pos;
            T[1] = (uint32_t)last;
            T[2] = (uint32_t)nmem;
            T[3] = 0;
        }
    }
    for (int k = k0; k < M; k += kstep) {
        const uint32_t key = valid ? rec[(size_t)e * MP + k] : 0xffffffffu;
        // rank among the block's keys (ties by lane); uniform lane reads
        // (v_readlane) instead of 64 dependent LDS permutes
        uint32_t rank = 0;
#pragma unroll
        for (int m = 0; m < kBlk; ++m) {
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)key, m);
            rank += (o < key || (o == key && m < l)) ? 1u : 0u;
        }
        T[blk_key_slot(k, (int)rank)] = key;
        inv[rank] = l;
        block_sync<kWaveSync>();
        const int mem = inv[l];
        const uint64_t bit = (mem < nmem) ? (1ull << mem) : 0ull;
        // prefix masks: members of ranks 0..l
        T[blk_mask_lo(k, l + 1)] = wave_inclusive_scan<true>((uint32_t)bit);
        T[blk_mask_hi(k, l + 1)] = wave_inclusive_scan<true>((uint32_t)(bit >> 32));
        if (l == 0) {
            T[blk_mask_lo(k, 0)] = 0u;
            T[blk_mask_hi(k, 0)] = 0u;
        }
        block_sync<kWaveSync>();
    }
}

// Table b of the list in global memory (see build_block_at).
template <int M, bool kWaveSync = false>
__device__ __forceinline__ void build_block(const uint32_t *__restrict__ rec, int32_t n,
                                            uint32_t *__restrict__ tabs, int32_t b, int32_t *inv,
                                            int k0 = 0, int kstep = 1) {
    build_block_at<M, kWaveSync>(rec, n, tabs + (size_t)b * blk_stride(M), b, inv, k0, kstep);
}

// Stage `nb` consecutive tables into LDS.
template <int M>
__device__ __forceinline__ void stage_tables(uint32_t *lds, const uint32_t *__restrict__ tabs,
                                             int32_t b0, int32_t nb) {
    constexpr int TS = blk_stride(M);
    const uint4 *src = reinterpret_cast<const uint4 *>(tabs + (size_t)b0 * TS);
    uint4 *dst = reinterpret_cast<uint4 *>(lds);
    const int nvec = nb * (TS / 4);
    for (int q = threadIdx.x; q < nvec; q += kFwdThreads) dst[q] = src[q];
}

// Forward: for each of the wave's kTJ x 64 points j (keys kj, run starts run),
// add the number of members of the staged blocks that dominate j.  With kOut,
// every dominating member also gains one in its 32-bit LDS counter oc[q]
// (member q = b * 64 + bit of the staged chunk): the same probes then give the
// out-degrees of the staged members, since every dominance pair (i before j's
// run) is probed exactly once.
template <int M, int TJ = kTJ, bool kOut = false>
__device__ __forceinline__ void fwd_blocks(const uint32_t *lt, int32_t nb, int32_t run_lo,
                                           int32_t run_hi, const uint32_t (&kj)[TJ][M],
                                           const int32_t (&run)[TJ], int32_t (&cnt)[TJ],
                                           uint32_t *oc = nullptr) {
    constexpr int TS = blk_stride(M);
    for (int32_t b = 0; b < nb; ++b) {
        const uint32_t *T = lt + b * TS;
        const int32_t bmin = (int32_t)T[0];
        const int32_t bmax = (int32_t)T[1];
        if (bmin >= run_hi) break;  // later blocks start later still
        const bool full = bmax < run_lo;
        // the TJ x M key searches in lockstep
        int ko[TJ * M];
        uint32_t x[TJ * M];
        uint64_t pm[TJ * M];
#pragma unroll
        for (int t = 0; t < TJ; ++t)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                ko[t * M + k] = k;
                x[t * M + k] = kj[t][k];
            }
        masks_many64<M, TJ * M, true>(T, ko, x, pm);
        uint64_t mt[TJ];
#pragma unroll
        for (int t = 0; t < TJ; ++t) {
            uint64_t m = ~0ull;
            if (!full) {
                if (run[t] <= bmin) m = 0ull;
                else if (run[t] <= bmax)
                    m = low_bits(count_pos_lt64(reinterpret_cast<const int32_t *>(T + blk_pos_off()),
                                                run[t]));
            }
#pragma unroll
            for (int k = 0; k < M; ++k) m &= pm[t * M + k];
            cnt[t] += __popcll(m);
            mt[t] = m;
        }
        if constexpr (kOut) {
            // one pass over the union of the lane's masks: a member that
            // dominates several of the lane's points is added once with their
            // number (the lane's points are neighbours in the sort, so they
            // share many dominators)
            uint32_t *ob = oc + b * kBlk;
            uint64_t u = 0ull;
#pragma unroll
            for (int t = 0; t < TJ; ++t) u |= mt[t];
            while (u) {
                const uint32_t bit = (uint32_t)__builtin_ctzll(u);
                uint32_t n = 0;
#pragma unroll
                for (int t = 0; t < TJ; ++t) n += (uint32_t)(mt[t] >> bit) & 1u;
                __hip_atomic_fetch_add(ob + bit, n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                u &= u - 1ull;
            }
        }
    }
}

// Loads the wave's points (records with MP stride, run starts) into registers.
template <int M, int TJ = kTJ>
__device__ __forceinline__ void load_points(const uint32_t *__restrict__ jrec,
                                            const int32_t *__restrict__ jrun, int32_t nj,
                                            int32_t jbase, int lane, uint32_t (&kj)[TJ][M],
                                            int32_t (&run)[TJ]) {
    constexpr int MP = rec_stride(M);
#pragma unroll
    for (int t = 0; t < TJ; ++t) {
        const int32_t q = jbase + t * kWave + lane;
        if (q < nj) {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = jrec[(size_t)q * MP + k];
            run[t] = jrun[q];
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = 0u;  // below every key: dominated by nothing
            run[t] = 0;
        }
    }
}


// Uniform reads of lists that other work-groups of a persistent launch may
// have written: a workgroup-scope atomic load is a vector load (never served by
// the scalar cache, which vector stores do not update).
template <typename T>
__device__ __forceinline__ T vld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// One item of a peeling level (Eq. (9)): the front blocks [b0, b0 + nb) (one
// chunk, staged in lt) against T consecutive tiles (kFwdThreads * TJ points
// each, TJ per lane) of the remaining list from tile jt0; every remaining point's count drops by the chunk members that
// dominate it.  The whole work-group (kFwdThreads) calls it with uniform
// arguments; it returns early, before any barrier, when every chunk member
// lies at or after the tiles' last run start.
template <int M, int T, int TJ = kTJ>
__device__ __forceinline__ void fwd_level_item(const uint32_t *__restrict__ tabs, int32_t b0,
                                               int32_t nb, const uint32_t *__restrict__ uk,
                                               const int32_t *__restrict__ urun, int32_t nu,
                                               int32_t *__restrict__ ucnt, int32_t jt0,
                                               uint32_t *lt) {
    constexpr int TS = blk_stride(M);
    if (jt0 * (kFwdThreads * TJ) >= nu) return;
    const int32_t tile_last = min((jt0 + T) * (kFwdThreads * TJ), nu) - 1;
    if ((int32_t)vld(&tabs[(size_t)b0 * TS]) >= vld(&urun[tile_last])) return;
    stage_tables<M>(lt, tabs, b0, nb);
    __syncthreads();
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int32_t jbase = (jt0 + t) * (kFwdThreads * TJ) + w * kWave * TJ;
        if (jbase >= nu) break;
        uint32_t kj[TJ][M];
        int32_t run[TJ], cnt[TJ];
        load_points<M, TJ>(uk, urun, nu, jbase, lane, kj, run);
#pragma unroll
        for (int u = 0; u < TJ; ++u) cnt[u] = 0;
        const int32_t run_lo = vld(&urun[jbase]);
        const int32_t run_hi = vld(&urun[min(jbase + kWave * TJ - 1, nu - 1)]);
        fwd_blocks<M, TJ>(lt, nb, run_lo, run_hi, kj, run, cnt);
#pragma unroll
        for (int u = 0; u < TJ; ++u) {
            const int32_t q = jbase + u * kWave + lane;
            if (q < nu && cnt[u]) atomicSub(&ucnt[q], cnt[u]);
        }
    }
}

// One tile of kFwdThreads * TJ remaining points against ng consecutive chunks
// of cb front tables from block b0 on: the points' keys stay in registers
// while each chunk is staged in LDS in turn, and each point's decrement goes
// out with one atomic.  A chunk that starts at or after the tile's last run
// ends the sweep (later chunks start later still).
// kLds: the chunk's tables are built in LDS from the front's records fk (nf of
// them) instead of staged from tabs: for small fronts, whose few tables cost
// less to rebuild per item than a launch of their own.  (A variant of its
// own: the build code needs far more registers than the probe.)
template <int M, int TJ, bool kLds>
__device__ __forceinline__ void fwd_level_group(const uint32_t *__restrict__ tabs, int32_t b0,
                                                int32_t cb, int32_t ng, int32_t nblk,
                                                const uint32_t *__restrict__ uk,
                                                const int32_t *__restrict__ urun, int32_t nu,
                                                int32_t *__restrict__ ucnt, int32_t jt,
                                                uint32_t *lt, const uint32_t *__restrict__ fk,
                                                int32_t nf, int32_t *inv /* [waves][kBlk] */) {
    constexpr int TS = blk_stride(M);
    constexpr int MP = rec_stride(M);
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
        // sorted position of the chunk's first member
        const int32_t first = kLds ? (int32_t)vld(&fk[(size_t)bs * kBlk * MP + M])
                                   : (int32_t)vld(&tabs[(size_t)bs * TS]);
        if (first >= last_run) break;
        const int32_t nb = min(cb, nblk - bs);
        __syncthreads();  // every wave is done with the previous chunk
        if constexpr (kLds) {
            // one (table, objective) per wave at a time; objective 0 also
            // writes the table's header and positions
            for (int job = w; job < nb * M; job += kFwdThreads / kWave)
                build_block_at<M, true>(fk, nf, lt + (job / M) * TS, bs + job / M,
                                        inv + w * kBlk, job % M, M);
        } else {
            stage_tables<M>(lt, tabs, bs, nb);
        }
        __syncthreads();
        if (active) fwd_blocks<M, TJ>(lt, nb, run_lo, run_hi, kj, run, cnt);
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
