// Block-bitset dominance kernels (see bitdom.h): table construction, the
// forward pass (each lane a later point j; counts the members of earlier
// blocks that dominate j -- in-degrees, or the peeling decrements of one
// front) and the backward pass (each lane an earlier point i; counts the
// members of later blocks that i dominates -- out-degrees).
//
// Dominance is Listing 1 / Eq. (6) on order keys (minimisation).  Candidates
// are restricted by the presort: an earlier point i can dominate j only when
// i lies before the run of points sharing j's key sum (identical rows and
// equal-sum points never dominate each other).
#include "bitdom.h"
#include "bitdom_wide.h"
#include "engine.h"
#include "kernels.h"
#include "prims.h"

namespace nsga3 {

// Block tables of a list of n records (n_static, or *n_dev when n_static < 0):
// one table per work-group at a time, one wave per objective (a table's
// latency is that of one objective, which matters for the small fronts of
// late peeling levels).
template <int M>
__global__ __launch_bounds__(M * kWave) void k_build_blocks(
    const uint32_t *__restrict__ rec, int32_t n_static, const int32_t *__restrict__ n_dev,
    uint32_t *__restrict__ tabs, const DevScalars *__restrict__ sc) {
    __shared__ int32_t inv[M][kBlk];
    if (sc->err) return;
    const int32_t n = n_static >= 0 ? n_static : *n_dev;
    const int32_t nblk = (n + kBlk - 1) / kBlk;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (int32_t b = (int32_t)blockIdx.x; b < nblk; b += (int32_t)gridDim.x)
        build_block<M, true>(rec, n, tabs, b, inv[w], w, M);
}

inline unsigned build_grid(int64_t nblk) { return (unsigned)nblk; }

// ---------------------------------------------------------------------------
// In-degrees over all points.  A work-group owns kTilesPerItem point tiles
// (their keys stay in registers) and sweeps kChunksPerItem consecutive block
// chunks, staging each in LDS once; its counts go out with one atomic per
// point.  Grid: x = tile group, y = chunk group, so neighbouring work-groups
// share their chunks in L2.  Chunks entirely after a tile's last run start
// are skipped.
// ---------------------------------------------------------------------------
// Tiles and chunks per count work-group: (tiles, chunks) = (2, 2) took
// 2.87 ms for both counts at N = 200k, M = 5; (4, 2) 3.01, (6, 2) 3.27,
// (1, 2) 2.92, (2, 1) 2.86, (2, 4) 2.93, (3, 2) 2.89, (4, 1) 2.97, (4, 3) 3.06.
constexpr int kTilesPerItem = 2;
constexpr int kChunksPerItem = 2;


// LDS out-degree counters of one staged chunk (one 32-bit counter per
// member) -> global (sorted positions b0 * 64 + member), cleared for the next
// chunk.
__device__ __forceinline__ void flush_out_counts(uint32_t *oc, int32_t b0, int32_t nb,
                                                 int32_t *__restrict__ dom_out) {
    for (int q = threadIdx.x; q < nb * kBlk; q += kFwdThreads) {
        const uint32_t v = oc[q];
        if (v) {
            atomicAdd(&dom_out[b0 * kBlk + q], (int32_t)v);
            oc[q] = 0u;
        }
    }
}

// kOut: out-degrees of the chunk members from the same probes (32-bit LDS
// counters oc[count_chunk * 64]; one global atomic per non-zero counter per
// chunk).
template <int M, bool kOut>
__device__ __forceinline__ void fwd_all_item(const uint32_t *__restrict__ tabs, int32_t nblk,
                                             const uint32_t *__restrict__ recs,
                                             const int32_t *__restrict__ runstart, int32_t N,
                                             int32_t *__restrict__ dom_in,
                                             int32_t *__restrict__ dom_out, int32_t jg, int32_t cg,
                                             uint32_t *lt, uint32_t *oc) {
    constexpr int CB = count_chunk<M>();
    constexpr int T = kTilesPerItem;
    const int32_t nIC = (nblk + CB - 1) / CB;
    const int32_t jt0 = jg * T;
    const int32_t c0 = cg * kChunksPerItem;
    const int32_t c1 = min(c0 + kChunksPerItem, nIC);
    if (c0 >= nIC) return;
    const int32_t last_run = runstart[min((jt0 + T) * kTileJ, N) - 1];
    if (c0 * CB * kBlk >= last_run) return;  // every chunk starts after every run
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    uint32_t kj[T][kTJ][M];
    int32_t run[T][kTJ], cnt[T][kTJ], run_lo[T], run_hi[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int32_t jbase = (jt0 + t) * kTileJ + w * kWave * kTJ;
        load_points<M>(recs, runstart, N, jbase, lane, kj[t], run[t]);
#pragma unroll
        for (int u = 0; u < kTJ; ++u) cnt[t][u] = 0;
        const int32_t jb = min(jbase, N - 1);
        run_lo[t] = __builtin_amdgcn_readfirstlane(runstart[jb]);
        run_hi[t] = jbase < N ? __builtin_amdgcn_readfirstlane(
                                    runstart[min(jbase + kWave * kTJ - 1, N - 1)])
                              : 0;  // no points: no chunk reaches them
    }
    if constexpr (kOut)
        for (int q = threadIdx.x; q < CB * kBlk; q += kFwdThreads) oc[q] = 0u;
    int32_t pb0 = -1, pnb = 0;  // chunk whose out-degree counters are pending
    for (int32_t c = c0; c < c1; ++c) {
        const int32_t b0 = c * CB;
        if (b0 * kBlk >= last_run) break;  // later chunks start later still
        const int32_t nb = min(CB, nblk - b0);
        __syncthreads();  // the previous chunk is consumed
        if constexpr (kOut)
            if (pb0 >= 0) flush_out_counts(oc, pb0, pnb, dom_out);
        stage_tables<M>(lt, tabs, b0, nb);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T; ++t)
            if (b0 * kBlk < run_hi[t])
                fwd_blocks<M, kTJ, kOut>(lt, nb, run_lo[t], run_hi[t], kj[t], run[t], cnt[t], oc);
        pb0 = b0;
        pnb = nb;
    }
    if constexpr (kOut) {
        if (pb0 >= 0) {
            __syncthreads();
            flush_out_counts(oc, pb0, pnb, dom_out);
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int32_t q = (jt0 + t) * kTileJ + w * kWave * kTJ + u * kWave + lane;
            if (q < N && cnt[t][u]) atomicAdd(&dom_in[q], cnt[t][u]);
        }
    }
}

// kOut: in-degrees and out-degrees from one pass.
template <int M, bool kOut>
__global__ __launch_bounds__(kFwdThreads) void k_fwd_all(const uint32_t *__restrict__ tabs,
                                                         int32_t nblk,
                                                         const uint32_t *__restrict__ recs,
                                                         const int32_t *__restrict__ runstart,
                                                         int32_t N, int32_t *__restrict__ dom_in,
                                                         int32_t *__restrict__ dom_out,
                                                         const DevScalars *__restrict__ sc) {
    __shared__ __attribute__((aligned(16))) uint32_t lt[count_chunk<M>() * blk_stride(M)];
    __shared__ uint32_t oc[kOut ? count_chunk<M>() * kBlk : 1];
    if (sc->err) return;
    fwd_all_item<M, kOut>(tabs, nblk, recs, runstart, N, dom_in, dom_out, (int32_t)blockIdx.x,
                          (int32_t)blockIdx.y, lt, oc);
}

// ---------------------------------------------------------------------------
// All-pairs counts with wide (128-member) tables, 4 <= M <= 10: the shape of
// fwd_all_item with a chunk of two wide tables and two point tiles per
// work-group (N = 200k, M = 5, both counts: 1.212 ms; two chunks 1.229, three
// 1.250, four 1.272; one tile and two or four chunks 1.29; three tiles and two
// chunks 1.23; chunks of one table, six per item 1.272; of three, two 1.406).
// ---------------------------------------------------------------------------
constexpr int kLdsCountWideDwords = 8192;
constexpr int kChunksPerItemWide = 1;
constexpr int kTilesPerItemWide = 2;
template <int M>
__host__ __device__ constexpr int count_chunk_wide() {
    return kLdsCountWideDwords / wblk_stride(M) < 1 ? 1 : kLdsCountWideDwords / wblk_stride(M);
}

// Wide tables of a list of n records (n_static, or *n_dev when n_static < 0).
template <int M>
__global__ __launch_bounds__(M * kWave) void k_build_wide(const uint32_t *__restrict__ rec,
                                                           int32_t n_static,
                                                           const int32_t *__restrict__ n_dev,
                                                           uint32_t *__restrict__ tabs,
                                                           const DevScalars *__restrict__ sc) {
    __shared__ int32_t inv[M][kWBlk];
    if (sc->err) return;
    const int32_t n = n_static >= 0 ? n_static : *n_dev;
    const int32_t nblk = (n + kWBlk - 1) / kWBlk;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (int32_t b = (int32_t)blockIdx.x; b < nblk; b += (int32_t)gridDim.x)
        build_wide_at<M>(rec, n, tabs + (size_t)b * wblk_stride(M), b, inv[w], w, M);
}

__device__ __forceinline__ void stage_words(uint32_t *lds, const uint32_t *__restrict__ src,
                                            int32_t nwords) {
    const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
    uint4 *d4 = reinterpret_cast<uint4 *>(lds);
    for (int q = threadIdx.x; q < nwords / 4; q += kFwdThreads) d4[q] = s4[q];
}

// One work item of the all-pairs counts over wide tables: kTilesPerItemWide
// tiles of points (group jg) against kChunksPerItemWide chunks of tables
// (group cg).  lt holds a chunk of tables, oc its out-degree counters.
template <int M, bool kOut>
__device__ __forceinline__ void fwd_all_wide_item(
    const uint32_t *__restrict__ tabs, int32_t nblk, const uint32_t *__restrict__ recs,
    const int32_t *__restrict__ runstart, int32_t N, int32_t *__restrict__ dom_in,
    int32_t *__restrict__ dom_out, int32_t jg, int32_t cg, uint32_t *lt, uint32_t *oc) {
    constexpr int CB = count_chunk_wide<M>();
    constexpr int TS = wblk_stride(M);
    constexpr int T = kTilesPerItemWide;
    const int32_t nIC = (nblk + CB - 1) / CB;
    const int32_t jt0 = jg * T;
    const int32_t c0 = cg * kChunksPerItemWide;
    const int32_t c1 = min(c0 + kChunksPerItemWide, nIC);
    if (c0 >= nIC) return;
    const int32_t last_run = runstart[min((jt0 + T) * kTileJ, N) - 1];
    if (c0 * CB * kWBlk >= last_run) return;  // every chunk starts after every run
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    uint32_t kj[T][kTJ][M];
    int32_t run[T][kTJ], cnt[T][kTJ], run_lo[T], run_hi[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int32_t jbase = (jt0 + t) * kTileJ + w * kWave * kTJ;
        load_points<M>(recs, runstart, N, jbase, lane, kj[t], run[t]);
#pragma unroll
        for (int u = 0; u < kTJ; ++u) cnt[t][u] = 0;
        const int32_t jb = min(jbase, N - 1);
        run_lo[t] = __builtin_amdgcn_readfirstlane(runstart[jb]);
        run_hi[t] = jbase < N ? __builtin_amdgcn_readfirstlane(
                                    runstart[min(jbase + kWave * kTJ - 1, N - 1)])
                              : 0;  // no points: no chunk reaches them
    }
    if constexpr (kOut)
        for (int q = threadIdx.x; q < CB * kWBlk; q += kFwdThreads) oc[q] = 0u;
    int32_t pb0 = -1, pnb = 0;  // chunk whose out-degree counters are pending
    for (int32_t c = c0; c < c1; ++c) {
        const int32_t b0 = c * CB;
        if (b0 * kWBlk >= last_run) break;  // later chunks start later still
        const int32_t nb = min(CB, nblk - b0);
        __syncthreads();  // the previous chunk is consumed
        if constexpr (kOut) {
            if (pb0 >= 0) {
                for (int q = threadIdx.x; q < pnb * kWBlk; q += kFwdThreads) {
                    const uint32_t v = oc[q];
                    if (v) {
                        atomicAdd(&dom_out[pb0 * kWBlk + q], (int32_t)v);
                        oc[q] = 0u;
                    }
                }
            }
        }
        stage_words(lt, tabs + (size_t)b0 * TS, nb * TS);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T; ++t)
            if (b0 * kWBlk < run_hi[t])
                fwd_blocks_wide<M, kTJ, kOut>(lt, nb, run_lo[t], run_hi[t], kj[t], run[t], cnt[t],
                                              oc);
        pb0 = b0;
        pnb = nb;
    }
    if constexpr (kOut) {
        if (pb0 >= 0) {
            __syncthreads();
            for (int q = threadIdx.x; q < pnb * kWBlk; q += kFwdThreads) {
                const uint32_t v = oc[q];
                if (v) atomicAdd(&dom_out[pb0 * kWBlk + q], (int32_t)v);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int32_t q = (jt0 + t) * kTileJ + w * kWave * kTJ + u * kWave + lane;
            if (q < N && cnt[t][u]) atomicAdd(&dom_in[q], cnt[t][u]);
        }
    }
}

template <int M, bool kOut>
__global__ __launch_bounds__(kFwdThreads) void k_fwd_all_wide(
    const uint32_t *__restrict__ tabs, int32_t nblk, const uint32_t *__restrict__ recs,
    const int32_t *__restrict__ runstart, int32_t N, int32_t *__restrict__ dom_in,
    int32_t *__restrict__ dom_out, const DevScalars *__restrict__ sc) {
    __shared__ __attribute__((aligned(16))) uint32_t lt[count_chunk_wide<M>() * wblk_stride(M)];
    __shared__ uint32_t oc[kOut ? count_chunk_wide<M>() * kWBlk : 1];
    if (sc->err) return;
    fwd_all_wide_item<M, kOut>(tabs, nblk, recs, runstart, N, dom_in, dom_out, (int32_t)blockIdx.x,
                               (int32_t)blockIdx.y, lt, oc);
}

// ---------------------------------------------------------------------------
// Peeling decrements of one level: blocks of the front F_k against the
// unranked list U_k.  Sizes come from the device; work items are handed out
// by block index first, then by a counter.
// ---------------------------------------------------------------------------
constexpr int kFwdLevelTiles = 1;  // remaining-list tiles per item (2 and 4 measured slower)
// Points per lane of the level kernel: 3 took the peel at N = 200k, M = 5 from
// 1.64 to 1.57 ms when it was measured (the all-pairs counts keep kTJ = 2,
// their best).
constexpr int kLevelTJ = 3;
constexpr int kLevelTileJ = kFwdThreads * kLevelTJ;
// Chunks of front tables a level work item sweeps for its tile (fewer on
// levels whose items would not fill two rounds of the grid): 2 took the peel
// at N = 200k, M = 5 from 1.127 to 1.115 ms, 4 to 1.16.
#ifndef NSGA3_LEVEL_CHUNKS
#define NSGA3_LEVEL_CHUNKS 2
#endif
constexpr int kLevelChunksPerItem = NSGA3_LEVEL_CHUNKS;

// kLds: the front's tables are built in LDS by every item from the front's
// records fk (no table-build launch for the level).
template <int M, bool kLds>
__global__ __launch_bounds__(kFwdThreads) void k_fwd_level(
    const uint32_t *__restrict__ tabs, const uint32_t *__restrict__ fk,
    const uint32_t *__restrict__ uk, const int32_t *__restrict__ urun,
    int32_t *__restrict__ ucnt, int32_t level, const int32_t *__restrict__ fsize,
    const int32_t *__restrict__ usize, uint32_t *__restrict__ work,
    const DevScalars *__restrict__ sc) {
    constexpr int TS = blk_stride(M);
    constexpr int CB = level_kernel_chunk<M>();
    __shared__ __attribute__((aligned(16))) uint32_t lt[CB * TS];
    __shared__ int32_t inv[kLds ? kFwdThreads / kWave * kBlk : 1];
    __shared__ int32_t s_item;
    if (sc->err) return;
    const int32_t nf = fsize[level];
    const int32_t nu = usize[level];
    if (nf == 0 || nu == 0) return;
    const int32_t nblk = (nf + kBlk - 1) / kBlk;
    constexpr int T = kFwdLevelTiles;
    static_assert(T == 1, "level items cover one remaining-list tile");
    const int32_t nJG = ((nu + kLevelTileJ - 1) / kLevelTileJ + T - 1) / T;
    // small levels: fewer tables per item while the items still fit in one
    // round of the grid (shorter items, same number of rounds)
    int32_t cb = CB;
    while (cb > 1 && (int64_t)((nblk + cb / 2 - 1) / (cb / 2)) * nJG <= (int64_t)gridDim.x) cb >>= 1;
    const int32_t nIC = (nblk + cb - 1) / cb;
    int32_t ng = kLevelChunksPerItem;
    while (ng > 1 && (int64_t)((nIC + ng - 1) / ng) * nJG < 2 * (int64_t)gridDim.x) ng >>= 1;
    const int64_t nitems = (int64_t)((nIC + ng - 1) / ng) * nJG;
    int64_t item = blockIdx.x;
    while (item < nitems) {
        const int32_t ig = (int32_t)(item / nJG);
        const int32_t jg = (int32_t)(item % nJG);
        fwd_level_group<M, kLevelTJ, kLds>(tabs, ig * ng * cb, cb, ng, nblk, uk, urun, nu, ucnt,
                                           jg, lt, fk, nf, inv);
        if (threadIdx.x == 0) s_item = (int32_t)(gridDim.x + atomicAdd(&work[level], 1u));
        __syncthreads();  // every wave is done with lt
        item = s_item;
        __syncthreads();
    }
}

// Decrements of one level against wide (128-member) tables of the front: the
// loop of k_fwd_level with wide chunks (two tables; 27 KiB of LDS at M = 5).
constexpr int kLdsLevelWideDwords = 6864;
constexpr int kLevelTJWide = 2;  // points per lane (three need 109 VGPRs)
constexpr int kLevelTileJWide = kFwdThreads * kLevelTJWide;
template <int M>
__host__ __device__ constexpr int level_wide_chunk() {
    return kLdsLevelWideDwords / wblk_stride(M) < 1 ? 1 : kLdsLevelWideDwords / wblk_stride(M);
}

template <int M>
__global__ __launch_bounds__(kFwdThreads) void k_fwd_level_wide(
    const uint32_t *__restrict__ tabs, const uint32_t *__restrict__ uk,
    const int32_t *__restrict__ urun, int32_t *__restrict__ ucnt, int32_t level,
    const int32_t *__restrict__ fsize, const int32_t *__restrict__ usize,
    uint32_t *__restrict__ work, const DevScalars *__restrict__ sc) {
    constexpr int TS = wblk_stride(M);
    constexpr int CB = level_wide_chunk<M>();
    __shared__ __attribute__((aligned(16))) uint32_t lt[CB * TS];
    __shared__ int32_t s_item;
    if (sc->err) return;
    const int32_t nf = fsize[level];
    const int32_t nu = usize[level];
    if (nf == 0 || nu == 0) return;
    const int32_t nblk = (nf + kWBlk - 1) / kWBlk;
    const int32_t nJG = (nu + kLevelTileJWide - 1) / kLevelTileJWide;
    int32_t cb = CB;
    while (cb > 1 && (int64_t)((nblk + cb / 2 - 1) / (cb / 2)) * nJG <= (int64_t)gridDim.x) cb >>= 1;
    const int32_t nIC = (nblk + cb - 1) / cb;
    int32_t ng = kLevelChunksPerItem;
    while (ng > 1 && (int64_t)((nIC + ng - 1) / ng) * nJG < 2 * (int64_t)gridDim.x) ng >>= 1;
    const int64_t nitems = (int64_t)((nIC + ng - 1) / ng) * nJG;
    int64_t item = blockIdx.x;
    while (item < nitems) {
        const int32_t ig = (int32_t)(item / nJG);
        const int32_t jg = (int32_t)(item % nJG);
        fwd_level_group_wide<M, kLevelTJWide>(tabs, ig * ng * cb, cb, ng, nblk, uk, urun, nu, ucnt, jg,
                                          lt);
        if (threadIdx.x == 0) s_item = (int32_t)(gridDim.x + atomicAdd(&work[level], 1u));
        __syncthreads();  // every wave is done with lt
        item = s_item;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Out-degrees over all points: each lane an earlier point i, later blocks;
// members j count when every key of j is >= i's and j lies in a later run
// (position >= runend(i)).
// ---------------------------------------------------------------------------
// Backward probe of the staged blocks for one group of kTJ earlier points per
// lane: members j with every key >= i's and a position >= runend(i).
template <int M>
__device__ __forceinline__ void bwd_blocks(const uint32_t *lt, int32_t nb, int32_t rend_lo,
                                           int32_t rend_hi, const uint32_t (&ki)[kTJ][M],
                                           const int32_t (&rend)[kTJ], int32_t (&cnt)[kTJ]) {
    constexpr int TS = blk_stride(M);
    for (int32_t b = 0; b < nb; ++b) {
        const uint32_t *T = lt + b * TS;
        const int32_t bmin = (int32_t)T[0];
        const int32_t bmax = (int32_t)T[1];
        if (bmax < rend_lo) continue;  // the whole block precedes every run end
        const uint64_t members = low_bits(T[2]);
        const bool full = bmin >= rend_hi;
        int ko[kTJ * M];
        uint32_t x[kTJ * M];
        uint64_t pm[kTJ * M];
#pragma unroll
        for (int t = 0; t < kTJ; ++t)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                ko[t * M + k] = k;
                x[t * M + k] = ki[t][k];
            }
        masks_many64<M, kTJ * M, false>(T, ko, x, pm);
#pragma unroll
        for (int t = 0; t < kTJ; ++t) {
            uint64_t m = members;
            if (!full) {
                if (rend[t] > bmax) m = 0ull;
                else if (rend[t] > bmin)
                    m &= ~low_bits(count_pos_lt64(reinterpret_cast<const int32_t *>(T + blk_pos_off()),
                                                  rend[t]));
            }
#pragma unroll
            for (int k = 0; k < M; ++k) m &= ~pm[t * M + k];
            cnt[t] += __popcll(m);
        }
    }
}

// Out-degrees over all points: each lane an earlier point i, later blocks;
// same work-group shape as the in-degree kernel.
template <int M>
__device__ __forceinline__ void bwd_all_item(const uint32_t *__restrict__ tabs, int32_t nblk,
                                             const uint32_t *__restrict__ recs,
                                             const int32_t *__restrict__ runend, int32_t N,
                                             int32_t *__restrict__ dom_out, int32_t jg, int32_t cg,
                                             uint32_t *lt) {
    constexpr int CB = count_chunk<M>();
    constexpr int MP = rec_stride(M);
    constexpr int T = kTilesPerItem;
    const int32_t nIC = (nblk + CB - 1) / CB;
    const int32_t it0 = jg * T;
    const int32_t c0 = cg * kChunksPerItem;
    const int32_t c1 = min(c0 + kChunksPerItem, nIC);
    if (c0 >= nIC || it0 * kTileJ >= N) return;
    const int32_t first_end = runend[it0 * kTileJ];  // smallest run end of the group
    if (min(c1 * CB * kBlk, N) - 1 < first_end) return;  // every member precedes every run end
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    uint32_t ki[T][kTJ][M];
    int32_t rend[T][kTJ], cnt[T][kTJ], rend_lo[T], rend_hi[T];
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int32_t ibase = (it0 + t) * kTileJ + w * kWave * kTJ;
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int32_t q = ibase + u * kWave + lane;
            cnt[t][u] = 0;
            if (q < N) {
#pragma unroll
                for (int k = 0; k < M; ++k) ki[t][u][k] = recs[(size_t)q * MP + k];
                rend[t][u] = runend[q];
            } else {
#pragma unroll
                for (int k = 0; k < M; ++k) ki[t][u][k] = 0xffffffffu;
                rend[t][u] = 0x7fffffff;  // dominates nothing
            }
        }
        if (ibase < N) {
            rend_lo[t] = __builtin_amdgcn_readfirstlane(runend[ibase]);
            rend_hi[t] = __builtin_amdgcn_readfirstlane(runend[min(ibase + kWave * kTJ - 1, N - 1)]);
        } else {
            rend_lo[t] = 0x7fffffff;  // no points: every block precedes
            rend_hi[t] = 0x7fffffff;
        }
    }
    for (int32_t c = c0; c < c1; ++c) {
        const int32_t b0 = c * CB;
        const int32_t nb = min(CB, nblk - b0);
        const int32_t chunk_last = min((b0 + nb) * kBlk, N) - 1;
        if (chunk_last < first_end) continue;  // precedes every run end of the group
        __syncthreads();  // the previous chunk is consumed
        stage_tables<M>(lt, tabs, b0, nb);
        __syncthreads();
#pragma unroll
        for (int t = 0; t < T; ++t)
            if (chunk_last >= rend_lo[t]) bwd_blocks<M>(lt, nb, rend_lo[t], rend_hi[t], ki[t], rend[t], cnt[t]);
    }
#pragma unroll
    for (int t = 0; t < T; ++t) {
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int32_t q = (it0 + t) * kTileJ + w * kWave * kTJ + u * kWave + lane;
            if (q < N && cnt[t][u]) atomicAdd(&dom_out[q], cnt[t][u]);
        }
    }
}

template <int M>
__global__ __launch_bounds__(kFwdThreads) void k_bwd_all(const uint32_t *__restrict__ tabs,
                                                         int32_t nblk,
                                                         const uint32_t *__restrict__ recs,
                                                         const int32_t *__restrict__ runend,
                                                         int32_t N, int32_t *__restrict__ dom_out,
                                                         const DevScalars *__restrict__ sc) {
    __shared__ __attribute__((aligned(16))) uint32_t lt[count_chunk<M>() * blk_stride(M)];
    if (sc->err) return;
    bwd_all_item<M>(tabs, nblk, recs, runend, N, dom_out, (int32_t)blockIdx.x, (int32_t)blockIdx.y, lt);
}

// ---------------------------------------------------------------------------
// Batched form for the engine's parked instances (one map entry per
// work-group; instances that finished early are skipped).
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T *inst_at(const EInst &I, size_t off) {
    return reinterpret_cast<T *>(I.ws + off);
}

// One table per work-group, one wave per objective (as k_build_blocks).
template <int M>
__global__ __launch_bounds__(M * kWave) void k_eng_build(const EInst *__restrict__ inst,
                                                         const EState *__restrict__ st,
                                                         const int2 *__restrict__ map) {
    __shared__ int32_t inv[M][kBlk];
    const int2 e = map[blockIdx.x];
    if (st[e.x].stage != kSDom) return;
    const EInst &I = inst[e.x];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    build_block<M, true>(inst_at<const uint32_t>(I, I.L.recs), I.N, inst_at<uint32_t>(I, I.L.tabs),
                         e.y, inv[w], w, M);
}

// kWhat: 0 in-degrees, 1 out-degrees (backward pass), 2 both from one pass.
template <int M, int kWhat>
__global__ __launch_bounds__(kFwdThreads) void k_eng_count(const EInst *__restrict__ inst,
                                                           const EState *__restrict__ st,
                                                           const int2 *__restrict__ map) {
    constexpr int CB = count_chunk<M>();
    __shared__ __attribute__((aligned(16))) uint32_t lt[CB * blk_stride(M)];
    __shared__ uint32_t oc[kWhat == 2 ? CB * kBlk : 1];
    const int2 e = map[blockIdx.x];
    if (st[e.x].stage != kSDom) return;
    const EInst &I = inst[e.x];
    const int32_t N = I.N;
    const int32_t nblk = (N + kBlk - 1) / kBlk;
    const int32_t nCG = ((nblk + CB - 1) / CB + kChunksPerItem - 1) / kChunksPerItem;
    const int32_t jg = e.y / nCG, cg = e.y % nCG;
    const uint32_t *tabs = inst_at<const uint32_t>(I, I.L.tabs);
    const uint32_t *recs = inst_at<const uint32_t>(I, I.L.recs);
    if (kWhat == 1)
        bwd_all_item<M>(tabs, nblk, recs, inst_at<const int32_t>(I, I.L.runend), N,
                        inst_at<int32_t>(I, I.L.dout), jg, cg, lt);
    else
        fwd_all_item<M, kWhat == 2>(tabs, nblk, recs, inst_at<const int32_t>(I, I.L.runstart), N,
                                    inst_at<int32_t>(I, I.L.din), inst_at<int32_t>(I, I.L.dout), jg,
                                    cg, lt, oc);
}

// Wide-table form (both counts from one pass), for the objective counts the
// single-selection counts also run on wide tables.
template <int M>
__global__ __launch_bounds__(M * kWave) void k_eng_build_wide(const EInst *__restrict__ inst,
                                                              const EState *__restrict__ st,
                                                              const int2 *__restrict__ map) {
    __shared__ int32_t inv[M][kWBlk];
    const int2 e = map[blockIdx.x];
    if (st[e.x].stage != kSDom) return;
    const EInst &I = inst[e.x];
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    build_wide_at<M>(inst_at<const uint32_t>(I, I.L.recs), I.N,
                     inst_at<uint32_t>(I, I.L.tabs) + (size_t)e.y * wblk_stride(M), e.y, inv[w], w,
                     M);
}

template <int M>
__global__ __launch_bounds__(kFwdThreads) void k_eng_count_wide(const EInst *__restrict__ inst,
                                                                const EState *__restrict__ st,
                                                                const int2 *__restrict__ map) {
    constexpr int CB = count_chunk_wide<M>();
    __shared__ __attribute__((aligned(16))) uint32_t lt[CB * wblk_stride(M)];
    __shared__ uint32_t oc[CB * kWBlk];
    const int2 e = map[blockIdx.x];
    if (st[e.x].stage != kSDom) return;
    const EInst &I = inst[e.x];
    const int32_t N = I.N;
    const int32_t nw = (N + kWBlk - 1) / kWBlk;
    const int32_t nCG = ((nw + CB - 1) / CB + kChunksPerItemWide - 1) / kChunksPerItemWide;
    fwd_all_wide_item<M, true>(inst_at<const uint32_t>(I, I.L.tabs), nw,
                               inst_at<const uint32_t>(I, I.L.recs),
                               inst_at<const int32_t>(I, I.L.runstart), N,
                               inst_at<int32_t>(I, I.L.din), inst_at<int32_t>(I, I.L.dout),
                               e.y / nCG, e.y % nCG, lt, oc);
}

template <int M>
static hipError_t launch_eng_bitdom(const EInst *inst, const EState *st, const int2 *bmap,
                                    int64_t nb_build, const int2 *cmap, int64_t nb_count,
                                    bool fused, bool wide, hipStream_t s) {
    if constexpr (wide_counts(M)) {
        if (wide) {
            if (nb_build > 0)
                hipLaunchKernelGGL(k_eng_build_wide<M>, dim3((unsigned)nb_build), dim3(M * kWave),
                                   0, s, inst, st, bmap);
            if (nb_count > 0)
                hipLaunchKernelGGL(k_eng_count_wide<M>, dim3((unsigned)nb_count),
                                   dim3(kFwdThreads), 0, s, inst, st, cmap);
            return hipGetLastError();
        }
    }
    if (nb_build > 0)
        hipLaunchKernelGGL(k_eng_build<M>, dim3((unsigned)nb_build), dim3(M * kWave), 0, s, inst, st,
                           bmap);
    if (nb_count > 0) {
        if (fused) {  // in-degrees and out-degrees from one pass
            hipLaunchKernelGGL((k_eng_count<M, 2>), dim3((unsigned)nb_count), dim3(kFwdThreads), 0,
                               s, inst, st, cmap);
        } else {
            hipLaunchKernelGGL((k_eng_count<M, 0>), dim3((unsigned)nb_count), dim3(kFwdThreads), 0,
                               s, inst, st, cmap);
            hipLaunchKernelGGL((k_eng_count<M, 1>), dim3((unsigned)nb_count), dim3(kFwdThreads), 0,
                               s, inst, st, cmap);
        }
    }
    return hipGetLastError();
}

bool engine_counts_wide(int M, int out_mode, bool wide) {
    return wide && wide_counts(M) && fused_out_counts(M, out_mode);
}

hipError_t engine_bitdom_launch(int M, const EInst *inst, const EState *st, const int2 *bmap,
                                int64_t nb_build, const int2 *cmap, int64_t nb_count,
                                int out_mode, bool wide, hipStream_t s) {
    const bool fused = fused_out_counts(M, out_mode);
    wide = engine_counts_wide(M, out_mode, wide);
    switch (M) {
#define NSGA3_CASE(m) case m: return launch_eng_bitdom<m>(inst, st, bmap, nb_build, cmap, nb_count, fused, wide, s);
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
}

void engine_bitdom_items(int64_t N, int M, int out_mode, bool wide, int64_t *n_build,
                         int64_t *n_count) {
    if (engine_counts_wide(M, out_mode, wide)) {
        int cbw = 1;
        switch (M) {
#define NSGA3_CB(m) case m: cbw = count_chunk_wide<m>(); break;
            NSGA3_CB(4) NSGA3_CB(5) NSGA3_CB(6) NSGA3_CB(7) NSGA3_CB(8) NSGA3_CB(9) NSGA3_CB(10)
#undef NSGA3_CB
            default: break;
        }
        const int64_t nw = (N + kWBlk - 1) / kWBlk;
        const int64_t nJG = ((N + kTileJ - 1) / kTileJ + kTilesPerItemWide - 1) / kTilesPerItemWide;
        const int64_t nCG = ((nw + cbw - 1) / cbw + kChunksPerItemWide - 1) / kChunksPerItemWide;
        *n_build = nw;
        *n_count = nJG * nCG;
        return;
    }
    int cb = 1;
    switch (M) {
#define NSGA3_CB(m) case m: cb = count_chunk<m>(); break;
        NSGA3_CB(2) NSGA3_CB(3) NSGA3_CB(4) NSGA3_CB(5) NSGA3_CB(6) NSGA3_CB(7) NSGA3_CB(8)
        NSGA3_CB(9) NSGA3_CB(10) NSGA3_CB(11) NSGA3_CB(12) NSGA3_CB(13) NSGA3_CB(14) NSGA3_CB(15)
        NSGA3_CB(16)
#undef NSGA3_CB
        default: break;
    }
    const int64_t nblk = (N + kBlk - 1) / kBlk;
    const int64_t nJG = ((N + kTileJ - 1) / kTileJ + kTilesPerItem - 1) / kTilesPerItem;
    const int64_t nCG = ((nblk + cb - 1) / cb + kChunksPerItem - 1) / kChunksPerItem;
    *n_build = nblk;
    *n_count = nJG * nCG;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
// Counting the dominating members inside the in-degree probes costs one LDS
// atomic per dominance pair, in a loop as long as the wave's densest mask.
// With few objectives dominance is dense (M = 2: about half of all pairs;
// quantised M = 3 data: 6 %), and the backward pass is cheaper there; from
// M = 4 on the fused form wins (N = 200k, M = 5: both counts 2.86 -> 1.69 ms).
constexpr int kFusedOutMinM = 4;

bool fused_out_counts(int M, int out_mode) {
    return out_mode == 0 || (out_mode < 0 && M >= kFusedOutMinM);
}

bool counts_use_wide(const SortViews &v) {
    return v.wide && wide_counts(v.M) && (!v.dom_out || fused_out_counts(v.M, v.out_mode));
}

template <int M>
static hipError_t launch_counts(const SortViews &v, hipStream_t s) {
    const int32_t N = (int32_t)v.N;
    if constexpr (wide_counts(M)) {
        if (counts_use_wide(v)) {
            const int32_t nw = (N + kWBlk - 1) / kWBlk;
            constexpr int CBW = count_chunk_wide<M>();
            hipLaunchKernelGGL(k_build_wide<M>, dim3((unsigned)nw), dim3(M * kWave), 0, s, v.recs, N,
                               (const int32_t *)nullptr, v.tabs_all, v.sc);
            const unsigned nJG = (unsigned)(((N + kTileJ - 1) / kTileJ + kTilesPerItemWide - 1) /
                                            kTilesPerItemWide);
            const unsigned nCG = (unsigned)(((nw + CBW - 1) / CBW + kChunksPerItemWide - 1) /
                                            kChunksPerItemWide);
            if (v.dom_out)
                hipLaunchKernelGGL((k_fwd_all_wide<M, true>), dim3(nJG, nCG), dim3(kFwdThreads), 0,
                                   s, v.tabs_all, nw, v.recs, v.runstart, N, v.dom_in_s,
                                   v.dom_out_s, v.sc);
            else
                hipLaunchKernelGGL((k_fwd_all_wide<M, false>), dim3(nJG, nCG), dim3(kFwdThreads), 0,
                                   s, v.tabs_all, nw, v.recs, v.runstart, N, v.dom_in_s,
                                   v.dom_out_s, v.sc);
            return hipGetLastError();
        }
    }
    const int32_t nblk = (N + kBlk - 1) / kBlk;
    constexpr int CB = count_chunk<M>();
    hipLaunchKernelGGL(k_build_blocks<M>, dim3(build_grid(nblk)), dim3(M * kWave), 0, s, v.recs, N,
                       (const int32_t *)nullptr, v.tabs_all, v.sc);
    const unsigned nIC = (unsigned)((nblk + CB - 1) / CB);
    const unsigned nJT = (unsigned)((N + kTileJ - 1) / kTileJ);
    const unsigned nJG = (nJT + kTilesPerItem - 1) / kTilesPerItem;
    const unsigned nCG = (nIC + kChunksPerItem - 1) / kChunksPerItem;
    if (v.dom_out && !fused_out_counts(M, v.out_mode)) {
        hipLaunchKernelGGL((k_fwd_all<M, false>), dim3(nJG, nCG), dim3(kFwdThreads), 0, s,
                           v.tabs_all, nblk, v.recs, v.runstart, N, v.dom_in_s, v.dom_out_s, v.sc);
        hipLaunchKernelGGL(k_bwd_all<M>, dim3(nJG, nCG), dim3(kFwdThreads), 0, s, v.tabs_all, nblk,
                           v.recs, v.runend, N, v.dom_out_s, v.sc);
    } else if (v.dom_out) {
        hipLaunchKernelGGL((k_fwd_all<M, true>), dim3(nJG, nCG), dim3(kFwdThreads), 0, s,
                           v.tabs_all, nblk, v.recs, v.runstart, N, v.dom_in_s, v.dom_out_s, v.sc);
    } else {
        hipLaunchKernelGGL((k_fwd_all<M, false>), dim3(nJG, nCG), dim3(kFwdThreads), 0, s,
                           v.tabs_all, nblk, v.recs, v.runstart, N, v.dom_in_s, v.dom_out_s, v.sc);
    }
    return hipGetLastError();
}

template <int M>
static hipError_t launch_build_all(const SortViews &v, hipStream_t s) {
    const int32_t N = (int32_t)v.N;
    const int32_t nblk = (N + kBlk - 1) / kBlk;
    hipLaunchKernelGGL(k_build_blocks<M>, dim3(build_grid(nblk)), dim3(M * kWave), 0, s, v.recs,
                       N, (const int32_t *)nullptr, v.tabs_all, v.sc);
    return hipGetLastError();
}

hipError_t run_build_all_tables(const SortViews &v, hipStream_t s) {
    switch (v.M) {
#define NSGA3_CASE(m) case m: return launch_build_all<m>(v, s);
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
}

hipError_t run_bit_counts(const SortViews &v, hipStream_t s) {
    switch (v.M) {
#define NSGA3_CASE(m) case m: return launch_counts<m>(v, s);
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
}

template <int M>
static void launch_level(const SortViews &v, const uint32_t *fk, const uint32_t *uk,
                         const int32_t *urun, int32_t *ucnt, int level, unsigned grid,
                         int32_t f_expect, bool tables_in_lds, hipStream_t s) {
    const int32_t N = (int32_t)v.N;
    if constexpr (wide_counts(M)) {
        if (!tables_in_lds && v.wide_levels) {
            const int32_t nw_max = (N + kWBlk - 1) / kWBlk;
            int32_t bgrid = nw_max;
            if (f_expect > 0) bgrid = min(nw_max, (f_expect + kWBlk - 1) / kWBlk * 5 / 4 + 4);
            // the wide front tables go to the all-points table space, which the
            // counts no longer need (tabs_lvl is sized for 64-member tables)
            hipLaunchKernelGGL(k_build_wide<M>, dim3((unsigned)bgrid), dim3(M * kWave), 0, s, fk, -1,
                               v.fsize + level, v.tabs_all, v.sc);
            hipLaunchKernelGGL(k_fwd_level_wide<M>, dim3(grid), dim3(kFwdThreads), 0, s, v.tabs_all,
                               uk, urun, ucnt, level, v.fsize, v.usize, v.work, v.sc);
            return;
        }
    }
    const int32_t nblk_max = (N + kBlk - 1) / kBlk;
    if (!tables_in_lds) {
        // the front's size is on the device: size the build grid from the size
        // expected (the kernel strides over any larger front), else for every point
        int32_t bgrid = nblk_max;
        if (f_expect > 0) bgrid = min(nblk_max, (f_expect + kBlk - 1) / kBlk * 5 / 4 + 4);
        hipLaunchKernelGGL(k_build_blocks<M>, dim3(build_grid(bgrid)), dim3(M * kWave), 0, s, fk,
                           -1, v.fsize + level, v.tabs_lvl, v.sc);
    }
    if (tables_in_lds)
        hipLaunchKernelGGL((k_fwd_level<M, true>), dim3(grid), dim3(kFwdThreads), 0, s, v.tabs_lvl,
                           fk, uk, urun, ucnt, level, v.fsize, v.usize, v.work, v.sc);
    else
        hipLaunchKernelGGL((k_fwd_level<M, false>), dim3(grid), dim3(kFwdThreads), 0, s,
                           v.tabs_lvl, fk, uk, urun, ucnt, level, v.fsize, v.usize, v.work, v.sc);
}

void run_bit_level(const SortViews &v, const uint32_t *fk, const uint32_t *uk, const int32_t *urun,
                   int32_t *ucnt, int level, unsigned grid, int32_t f_expect,
                   bool tables_in_lds, hipStream_t s) {
    switch (v.M) {
#define NSGA3_CASE(m) \
    case m: launch_level<m>(v, fk, uk, urun, ucnt, level, grid, f_expect, tables_in_lds, s); break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: break;
    }
}

size_t level_tables_bytes(int64_t N, int M) {
    return (size_t)((N + kBlk - 1) / kBlk) * (size_t)blk_stride(M) * sizeof(uint32_t);
}

size_t bit_tables_bytes(int64_t N, int M) {
    const size_t narrow = (size_t)((N + kBlk - 1) / kBlk) * (size_t)blk_stride(M);
    const size_t wide = (size_t)((N + kWBlk - 1) / kWBlk) * (size_t)wblk_stride(M);
    return (narrow > wide ? narrow : wide) * sizeof(uint32_t);
}

}  // namespace nsga3
