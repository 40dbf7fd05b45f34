// Front peeling (Eq. (8)-(9), Alg. S.3) and the last admitted front (end of
// Sec. IV-A.1) on gfx950.
//
// State kept in sorted-position order, double buffered by level parity:
//   F_k: front-k records (keys + sorted position)
//   U_k: records of the points still unranked after level k, their run starts
//        and their remaining in-degree (number of unranked dominators).
// Level k:  split   -- U_{k-1} (level 0: every point, in-degree from the
//                      dominance counts) is divided into F_k (remaining
//                      in-degree 0, rank k) and U_k, both keeping order;
//           phase A -- every U_k point subtracts its number of dominators in
//                      F_k (only earlier positions can dominate).
// The host enqueues a number of levels taken from the previous call (each
// level is two ordinary launches that return at once when peeling is done);
// a cooperative tail kernel finishes any levels beyond them with grid
// barriers.  Front sizes go to fsize[k], remaining sizes to usize[k].
#include "kernels.h"
#include "prims.h"
#include "tile.h"

namespace nsga3 {

constexpr int kSplitItems = 2;
constexpr int kSplitTile = kThreads * kSplitItems;

// Look-back state word: [63:62] status (0 none, 1 aggregate, 2 inclusive),
// [61:31] front count, [30:0] remaining count.
__device__ __forceinline__ uint64_t lb_pack(uint32_t st, uint32_t f, uint32_t u) {
    return ((uint64_t)st << 62) | ((uint64_t)f << 31) | (uint64_t)u;
}

// Copies one record (MP dwords, 16-byte aligned).
template <int MP>
__device__ __forceinline__ void copy_rec(uint32_t *__restrict__ d, const uint32_t *__restrict__ s) {
#pragma unroll
    for (int k = 0; k < MP / 4; ++k)
        reinterpret_cast<uint4 *>(d)[k] = reinterpret_cast<const uint4 *>(s)[k];
}

// ---------------------------------------------------------------------------
// split (one launch per level): single-pass ordered partition with a
// decoupled look-back over per-block counts.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kThreads) void k_split(
    const uint32_t *__restrict__ srec, const int32_t *__restrict__ srun,
    const int32_t *__restrict__ scnt, int32_t n_static, int32_t level, uint32_t *__restrict__ fdst,
    uint32_t *__restrict__ udst, int32_t *__restrict__ urun_dst, int32_t *__restrict__ ucnt_dst,
    int32_t *__restrict__ rank_s, int32_t *__restrict__ fsize, int32_t *__restrict__ usize,
    uint64_t *__restrict__ lb_cur, uint64_t *__restrict__ lb_next, DevScalars *__restrict__ sc) {
    constexpr int MP = rec_stride(M);
    __shared__ uint32_t lds[17];
    __shared__ uint32_t s_pref[2];
    if (threadIdx.x == 0) lb_next[blockIdx.x] = 0;  // ready for the next level
    if (sc->err) return;
    const int32_t n = n_static >= 0 ? n_static : usize[level - 1];
    if (n_static < 0 && n > 0 && fsize[level - 1] == 0) {  // impossible for a partial order
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
        return;
    }
    if (n == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) { fsize[level] = 0; usize[level] = 0; }
        return;
    }
    const int32_t e0 = (int32_t)blockIdx.x * kSplitTile;
    if (e0 >= n) return;
    const int32_t nb = (n + kSplitTile - 1) / kSplitTile;
    // each thread owns kSplitItems consecutive elements
    const int32_t t0 = e0 + (int32_t)threadIdx.x * kSplitItems;
    uint32_t zf = 0, zu = 0;
    int32_t cnt[kSplitItems];
#pragma unroll
    for (int q = 0; q < kSplitItems; ++q) {
        const int32_t e = t0 + q;
        cnt[q] = e < n ? scnt[e] : -1;
        zf += cnt[q] == 0 ? 1u : 0u;
        zu += cnt[q] > 0 ? 1u : 0u;
    }
    uint32_t tot;
    const uint32_t ex = block_exclusive_scan((zf << 16) | zu, lds, &tot);
    if (threadIdx.x < kWave) {
        // look-back by the first wave: lane q reads the state of block
        // base - q, so one round covers 64 predecessors; the nearest block
        // with an inclusive prefix ends the walk (before block 0 the prefix
        // is 0), and every block nearer than it must have published its
        // aggregate, or the round is read again
        const uint32_t bf = tot >> 16, bu = tot & 0xffffu;
        const int lane = (int)lane_id();
        uint32_t pf = 0, pu = 0;
        if (blockIdx.x == 0) {
            if (lane == 0)
                __hip_atomic_store(&lb_cur[0], lb_pack(2, bf, bu), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            if (lane == 0)
                __hip_atomic_store(&lb_cur[blockIdx.x], lb_pack(1, bf, bu), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
            int32_t base = (int32_t)blockIdx.x - 1;
            uint64_t spins = 0;
            while (true) {
                const int32_t q = base - lane;
                const uint64_t v = q >= 0 ? __hip_atomic_load(&lb_cur[q], __ATOMIC_RELAXED,
                                                              __HIP_MEMORY_SCOPE_AGENT)
                                          : lb_pack(2, 0, 0);
                const uint32_t st = (uint32_t)(v >> 62);
                const uint64_t inc = ballot(st == 2);
                const int first = inc ? __builtin_ctzll(inc) : kWave;   // nearest inclusive lane
                const uint64_t need = first < kWave - 1 ? ((2ull << first) - 1ull) : ~0ull;
                if (ballot(st == 0) & need) {
                    __builtin_amdgcn_s_sleep(1);
                    if (++spins > (1ull << 26)) {  // a predecessor never published
                        if (lane == 0) atomicOr(&sc->err, (uint32_t)kErrBarrierTimeout);
                        break;
                    }
                    continue;
                }
                const bool take = lane <= first;
                pf += wave_sum(take ? (uint32_t)(v >> 31) & 0x7fffffffu : 0u);
                pu += wave_sum(take ? (uint32_t)v & 0x7fffffffu : 0u);
                if (inc) break;
                base -= kWave;
            }
            if (lane == 0)
                __hip_atomic_store(&lb_cur[blockIdx.x], lb_pack(2, pf + bf, pu + bu), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            s_pref[0] = pf;
            s_pref[1] = pu;
            if ((int32_t)blockIdx.x == nb - 1) {
                fsize[level] = (int32_t)(pf + bf);
                usize[level] = (int32_t)(pu + bu);
            }
        }
    }
    __syncthreads();
    uint32_t of = s_pref[0] + (ex >> 16);
    uint32_t ou = s_pref[1] + (ex & 0xffffu);
#pragma unroll
    for (int q = 0; q < kSplitItems; ++q) {
        const int32_t e = t0 + q;
        if (e >= n) break;
        const uint32_t *r = srec + (size_t)e * MP;
        if (cnt[q] == 0) {
            copy_rec<MP>(fdst + (size_t)of * MP, r);
            rank_s[r[M]] = level;
            ++of;
        } else {
            copy_rec<MP>(udst + (size_t)ou * MP, r);
            urun_dst[ou] = srun[e];
            ucnt_dst[ou] = cnt[q];
            ++ou;
        }
    }
}

// One wave's share of a phase-A work item: its kT * 64 unranked points
// against a chunk of front members staged in LDS.
template <int M>
__device__ __forceinline__ void pair_item(const uint32_t *lrec, int32_t nfi,
                                          const uint32_t *__restrict__ uk,
                                          const int32_t *__restrict__ urun,
                                          int32_t *__restrict__ ucnt, int32_t nu, int32_t jbase,
                                          int32_t qlast, int lane) {
    constexpr int MP = rec_stride(M);
    const int32_t run_hi = urun[qlast];
    const int32_t run_lo = urun[jbase];
    uint32_t kj[kT][M];
    int32_t run[kT], cin[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int32_t q = jbase + t * kWave + lane;
        cin[t] = 0;
        if (q < nu) {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = uk[(size_t)q * MP + k];
            run[t] = urun[q];
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = 0u;
            run[t] = 0;
        }
    }
    tile_rows_bounded<M>(lrec, nfi, run_lo, run_hi, kj, run, cin);
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int32_t q = jbase + t * kWave + lane;
        if (q < nu && cin[t]) atomicSub(&ucnt[q], cin[t]);
    }
}

// Front members per phase-A chunk: at most 16 KiB of records in LDS, fewer
// on small levels so that the level still spreads over many work items.
template <int M>
__device__ __forceinline__ int32_t phase_a_chunk(int32_t nf, int32_t nJT) {
    constexpr int kMaxIC = 4096 / rec_stride(M);
    int32_t ic = kMaxIC;
    while (ic > 64 && (int64_t)((nf + ic - 1) / ic) * nJT < 4096) ic >>= 1;
    return ic;
}

// ---------------------------------------------------------------------------
// phase A (one launch per level): F_k x U_k decrements.  Work item = (chunk of
// front members, tile of kJT unranked points); a block's first item is its
// index, later items come from a shared counter.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kThreads) void k_phase_a(
    const uint32_t *__restrict__ fk, const uint32_t *__restrict__ uk,
    const int32_t *__restrict__ urun, int32_t *__restrict__ ucnt, int32_t level,
    const int32_t *__restrict__ fsize, const int32_t *__restrict__ usize,
    uint32_t *__restrict__ work, const DevScalars *__restrict__ sc) {
    constexpr int MP = rec_stride(M);
    __shared__ __attribute__((aligned(16))) uint32_t lrec[4096];
    __shared__ int32_t s_item;
    if (sc->err) return;
    const int32_t nf = fsize[level];
    const int32_t nu = usize[level];
    if (nf == 0 || nu == 0) return;
    const int32_t nJT = (nu + kJT - 1) / kJT;
    const int32_t IC = phase_a_chunk<M>(nf, nJT);
    const int32_t nIC = (nf + IC - 1) / IC;
    const int64_t nitems = (int64_t)nIC * nJT;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    int64_t item = blockIdx.x;
    while (item < nitems) {
        const int32_t ic = (int32_t)(item / nJT);
        const int32_t jt = (int32_t)(item % nJT);
        const int32_t f0 = ic * IC;
        const int32_t f1 = min(f0 + IC, nf);
        const int32_t tile_last = min(jt * kJT + kJT - 1, nu - 1);
        if ((int32_t)fk[(size_t)f0 * MP + M] < urun[tile_last]) {  // block-uniform
            {
                const uint4 *src = reinterpret_cast<const uint4 *>(fk + (size_t)f0 * MP);
                uint4 *dst = reinterpret_cast<uint4 *>(lrec);
                const int nvec = (f1 - f0) * (MP / 4);
                for (int q = threadIdx.x; q < nvec; q += kThreads) dst[q] = src[q];
            }
            __syncthreads();
            const int32_t jbase = jt * kJT + w * kWave * kT;
            if (jbase < nu)
                pair_item<M>(lrec, f1 - f0, uk, urun, ucnt, nu, jbase,
                             min(jbase + kWave * kT - 1, nu - 1), lane);
        }
        if (threadIdx.x == 0) s_item = (int32_t)(gridDim.x + atomicAdd(&work[level], 1u));
        __syncthreads();  // also: every wave is done with lrec
        item = s_item;
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Cooperative tail: levels k0, k0+1, ... with grid barriers, for populations
// with more fronts than the host enqueued.  Front chunks are staged in LDS
// because the front list is rewritten inside this kernel.
// ---------------------------------------------------------------------------
template <int M>
__device__ bool tail_split(const uint32_t *__restrict__ srec, const int32_t *__restrict__ srun,
                           const int32_t *__restrict__ scnt, int32_t n, uint32_t *__restrict__ fdst,
                           uint32_t *__restrict__ udst, int32_t *__restrict__ urun_dst,
                           int32_t *__restrict__ ucnt_dst, int32_t *__restrict__ rank_s,
                           int32_t level, uint32_t *__restrict__ blkcnt, DevScalars *__restrict__ sc,
                           GridBar *bar, int32_t *nf_out, int32_t *nu_out) {
    constexpr int MP = rec_stride(M);
    __shared__ uint32_t lds[17];
    __shared__ uint32_t red[4 * kWaves];
    const uint32_t G = gridDim.x;
    const int32_t seg = (int32_t)((n + (int64_t)G - 1) / G);
    const int32_t s0 = min((int32_t)blockIdx.x * seg, n);
    const int32_t s1 = min(s0 + seg, n);
    uint32_t nz = 0, nn = 0;
    for (int32_t e = s0 + threadIdx.x; e < s1; e += kThreads) {
        if (scnt[e] == 0) ++nz; else ++nn;
    }
    nz = wave_sum(nz);
    nn = wave_sum(nn);
    if (lane_id() == 0) {
        red[threadIdx.x / kWave] = nz;
        red[kWaves + threadIdx.x / kWave] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, c = 0;
        for (int q = 0; q < kWaves; ++q) { a += red[q]; c += red[kWaves + q]; }
        blkcnt[2 * blockIdx.x] = a;
        blkcnt[2 * blockIdx.x + 1] = c;
    }
    if (!grid_barrier2(bar, &sc->err)) return false;
    uint32_t pf = 0, pu = 0, tf = 0, tu = 0;
    for (uint32_t q = threadIdx.x; q < G; q += kThreads) {
        const uint32_t a = __hip_atomic_load(&blkcnt[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t c = __hip_atomic_load(&blkcnt[2 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tf += a; tu += c;
        if (q < blockIdx.x) { pf += a; pu += c; }
    }
    pf = wave_sum(pf); pu = wave_sum(pu); tf = wave_sum(tf); tu = wave_sum(tu);
    __syncthreads();
    if (lane_id() == 0) {
        const int w = threadIdx.x / kWave;
        red[w] = pf; red[kWaves + w] = pu; red[2 * kWaves + w] = tf; red[3 * kWaves + w] = tu;
    }
    __syncthreads();
    pf = pu = tf = tu = 0;
    for (int q = 0; q < kWaves; ++q) {
        pf += red[q]; pu += red[kWaves + q]; tf += red[2 * kWaves + q]; tu += red[3 * kWaves + q];
    }
    __syncthreads();
    for (int32_t base = s0; base < s1; base += kThreads) {
        const int32_t e = base + (int32_t)threadIdx.x;
        const bool valid = e < s1;
        const int32_t cnt = valid ? scnt[e] : 1;
        const uint32_t isf = (valid && cnt == 0) ? 1u : 0u;
        const uint32_t isu = (valid && cnt != 0) ? 1u : 0u;
        uint32_t totf, totu;
        const uint32_t exf = block_exclusive_scan(isf, lds, &totf);
        const uint32_t exu = block_exclusive_scan(isu, lds, &totu);
        if (valid) {
            const uint32_t *r = srec + (size_t)e * MP;
            if (isf) {
                copy_rec<MP>(fdst + (size_t)(pf + exf) * MP, r);
                rank_s[r[M]] = level;
            } else {
                const uint32_t slot = pu + exu;
                copy_rec<MP>(udst + (size_t)slot * MP, r);
                urun_dst[slot] = srun[e];
                ucnt_dst[slot] = cnt;
            }
        }
        pf += totf;
        pu += totu;
    }
    *nf_out = (int32_t)tf;
    *nu_out = (int32_t)tu;
    return true;
}

template <int M>
__device__ void tail_phase_a(const uint32_t *__restrict__ fk, int32_t nf,
                             const uint32_t *__restrict__ uk, const int32_t *__restrict__ urun,
                             int32_t *__restrict__ ucnt, int32_t nu, uint32_t *lrec,
                             int64_t item0, int64_t istride) {
    constexpr int MP = rec_stride(M);
    constexpr int IC = 8192 / MP;  // 32 KiB of records in LDS
    const int nIC = (nf + IC - 1) / IC;
    const int nJT = (nu + kJT - 1) / kJT;
    const int64_t nitems = (int64_t)nIC * nJT;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    for (int64_t item = item0; item < nitems; item += istride) {
        const int jt = (int)(item % nJT);
        const int ic = (int)(item / nJT);
        const int f0 = ic * IC;
        const int f1 = min(f0 + IC, nf);
        const int tile_last = min(jt * kJT + kJT - 1, nu - 1);
        if ((int)fk[(size_t)f0 * MP + M] >= urun[tile_last]) continue;  // block-uniform skip
        __syncthreads();
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(fk + (size_t)f0 * MP);
            uint4 *dst = reinterpret_cast<uint4 *>(lrec);
            const int nvec = (f1 - f0) * (MP / 4);
            for (int q = threadIdx.x; q < nvec; q += kThreads) dst[q] = src[q];
        }
        __syncthreads();
        const int jbase = jt * kJT + w * kWave * kT;
        if (jbase < nu) {
            uint32_t kj[kT][M];
            int32_t run[kT], cin[kT];
#pragma unroll
            for (int t = 0; t < kT; ++t) {
                const int q = jbase + t * kWave + lane;
                cin[t] = 0;
                if (q < nu) {
#pragma unroll
                    for (int k = 0; k < M; ++k) kj[t][k] = uk[(size_t)q * MP + k];
                    run[t] = urun[q];
                } else {
#pragma unroll
                    for (int k = 0; k < M; ++k) kj[t][k] = 0u;
                    run[t] = 0;
                }
            }
            const int qlast = min(jbase + kWave * kT - 1, nu - 1);
            const int run_lo = __builtin_amdgcn_readfirstlane(urun[jbase]);
            const int run_hi = __builtin_amdgcn_readfirstlane(urun[qlast]);
            tile_rows_bounded<M>(lrec, f1 - f0, run_lo, run_hi, kj, run, cin);
#pragma unroll
            for (int t = 0; t < kT; ++t) {
                const int q = jbase + t * kWave + lane;
                if (q < nu && cin[t]) atomicSub(&ucnt[q], cin[t]);
            }
        }
    }
}

// One work-group finishes the levels from `level` on (nu points unranked
// before it), with block barriers only: ordered split, then pairwise
// decrements of the remaining list by the new front.
template <int M>
__device__ void tail_levels_one_block(int32_t level, int32_t nu, uint32_t *__restrict__ fk0,
                                      uint32_t *__restrict__ fk1, uint32_t *__restrict__ uk0,
                                      uint32_t *__restrict__ uk1, int32_t *__restrict__ urun0,
                                      int32_t *__restrict__ urun1, int32_t *__restrict__ ucnt0,
                                      int32_t *__restrict__ ucnt1, int32_t *__restrict__ rank_s,
                                      int32_t *__restrict__ fsize, int32_t *__restrict__ usize,
                                      DevScalars *__restrict__ sc, uint32_t *lrec, uint32_t *lds) {
    constexpr int MP = rec_stride(M);
    for (;;) {
        const int p = (level - 1) & 1, q = level & 1;
        const uint32_t *us = p ? uk1 : uk0;
        const int32_t *rs = p ? urun1 : urun0;
        const int32_t *cs = p ? ucnt1 : ucnt0;
        uint32_t *fd = q ? fk1 : fk0;
        uint32_t *ud = q ? uk1 : uk0;
        int32_t *rd = q ? urun1 : urun0;
        int32_t *cd = q ? ucnt1 : ucnt0;
        // ordered split of U_{level-1}
        uint32_t of = 0, ou = 0;
        for (int32_t base = 0; base < nu; base += kThreads) {
            const int32_t e = base + (int32_t)threadIdx.x;
            const bool valid = e < nu;
            const int32_t cnt = valid ? cs[e] : 1;
            const uint32_t isf = (valid && cnt == 0) ? 1u : 0u;
            const uint32_t isu = (valid && cnt != 0) ? 1u : 0u;
            uint32_t totf, totu;
            const uint32_t exf = block_exclusive_scan(isf, lds, &totf);
            const uint32_t exu = block_exclusive_scan(isu, lds, &totu);
            if (valid) {
                const uint32_t *r = us + (size_t)e * MP;
                if (isf) {
                    copy_rec<MP>(fd + (size_t)(of + exf) * MP, r);
                    rank_s[r[M]] = level;
                } else {
                    copy_rec<MP>(ud + (size_t)(ou + exu) * MP, r);
                    rd[ou + exu] = rs[e];
                    cd[ou + exu] = cnt;
                }
            }
            of += totf;
            ou += totu;
        }
        if (threadIdx.x == 0) { fsize[level] = (int32_t)of; usize[level] = (int32_t)ou; }
        __syncthreads();
        if (ou == 0) return;
        if (of == 0) {
            if (threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
            return;
        }
        tail_phase_a<M>(fd, (int32_t)of, ud, rd, cd, (int32_t)ou, lrec, 0, 1);
        __syncthreads();
        nu = (int32_t)ou;
        ++level;
    }
}

template <int M>
__global__ __launch_bounds__(kThreads) void k_peel_tail(
    int32_t k0, uint32_t *__restrict__ fk0, uint32_t *__restrict__ fk1, uint32_t *__restrict__ uk0,
    uint32_t *__restrict__ uk1, int32_t *__restrict__ urun0, int32_t *__restrict__ urun1,
    int32_t *__restrict__ ucnt0, int32_t *__restrict__ ucnt1, int32_t *__restrict__ rank_s,
    int32_t *__restrict__ fsize, int32_t *__restrict__ usize, uint32_t *__restrict__ blkcnt,
    DevScalars *__restrict__ sc, GridBar *__restrict__ bar) {
    __shared__ __attribute__((aligned(16))) uint32_t lrec[8192];
    __shared__ uint32_t lds1[17];
    if (__hip_atomic_load(&sc->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    int32_t level = k0;
    int32_t nu = usize[level - 1];
    if (nu == 0) return;  // the enqueued levels finished peeling
    if (fsize[level - 1] == 0) {
        if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
        return;
    }
    if (nu <= kTailOneBlockMax) {  // few points left: one work-group, no grid barriers
        if (blockIdx.x == 0)
            tail_levels_one_block<M>(level, nu, fk0, fk1, uk0, uk1, urun0, urun1, ucnt0, ucnt1,
                                     rank_s, fsize, usize, sc, lrec, lds1);
        return;
    }
    for (;;) {
        const int p = (level - 1) & 1, q = level & 1;
        uint32_t *us = p ? uk1 : uk0;
        int32_t *rs = p ? urun1 : urun0;
        int32_t *cs = p ? ucnt1 : ucnt0;
        uint32_t *fd = q ? fk1 : fk0;
        uint32_t *ud = q ? uk1 : uk0;
        int32_t *rd = q ? urun1 : urun0;
        int32_t *cd = q ? ucnt1 : ucnt0;
        int32_t nf2 = 0, nu2 = 0;
        if (!tail_split<M>(us, rs, cs, nu, fd, ud, rd, cd, rank_s, level, blkcnt, sc, bar, &nf2, &nu2))
            return;
        if (blockIdx.x == 0 && threadIdx.x == 0) { fsize[level] = nf2; usize[level] = nu2; }
        if (!grid_barrier2(bar, &sc->err)) return;
        if (nu2 == 0) return;
        if (nf2 == 0) {  // impossible for a partial order; leave instead of spinning
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
            return;
        }
        tail_phase_a<M>(fd, nf2, ud, rd, cd, nu2, lrec, blockIdx.x, gridDim.x);
        if (!grid_barrier2(bar, &sc->err)) return;
        nu = nu2;
        ++level;
    }
}

// Single-workgroup tail (usable inside captured graphs, where cooperative
// launches are not): one block finishes the levels from k0 on.  Meant for the
// few points left after the enqueued levels.
template <int M>
__global__ __launch_bounds__(kThreads) void k_peel_tail_block(
    int32_t k0, uint32_t *__restrict__ fk0, uint32_t *__restrict__ fk1, uint32_t *__restrict__ uk0,
    uint32_t *__restrict__ uk1, int32_t *__restrict__ urun0, int32_t *__restrict__ urun1,
    int32_t *__restrict__ ucnt0, int32_t *__restrict__ ucnt1, int32_t *__restrict__ rank_s,
    int32_t *__restrict__ fsize, int32_t *__restrict__ usize, DevScalars *__restrict__ sc) {
    __shared__ __attribute__((aligned(16))) uint32_t lrec[8192];
    __shared__ uint32_t lds[17];
    if (sc->err) return;
    const int32_t nu = usize[k0 - 1];
    if (nu == 0) return;
    if (fsize[k0 - 1] == 0) {
        if (threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
        return;
    }
    tail_levels_one_block<M>(k0, nu, fk0, fk1, uk0, uk1, urun0, urun1, ucnt0, ucnt1, rank_s, fsize,
                             usize, sc, lrec, lds);
}

// a3: number of fronts and the last admitted front l = rank of the K-th
// smallest rank (0-based position K-1).
__global__ void k_last_front(const int32_t *__restrict__ fsize, const int32_t *__restrict__ usize,
                             int64_t N, int64_t K, DevScalars *__restrict__ sc) {
    if (threadIdx.x != 0 || sc->err) return;
    int32_t L = 0;
    for (int64_t k = 0; k < N; ++k) {
        L = (int32_t)k + 1;
        if (usize[k] == 0) break;
    }
    int64_t cum = 0;
    int32_t l = L - 1;
    for (int32_t k = 0; k < L; ++k) {
        if (cum + fsize[k] >= K) { l = k; break; }
        cum += fsize[k];
    }
    sc->num_fronts = L;
    // host feedback: the front count, then the points left after each level
    sc->fb[0] = L;
    for (int32_t k = 0; k < L && k < kProfLevels; ++k) sc->fb[1 + k] = usize[k];
    sc->last_front = l;
    sc->last_front_size = fsize[l];
    sc->n_before = cum;
    sc->num_from_last = K - cum;
}

template <int M>
static hipError_t launch_peel(const SortViews &v, const LaunchCfg &cfg, hipStream_t s) {
    const int32_t N = (int32_t)v.N;
    const unsigned nbs = (unsigned)((N + kSplitTile - 1) / kSplitTile);
    const int levels = cfg.host_levels < 1 ? 1 : cfg.host_levels;
    const unsigned ga = (unsigned)(cfg.num_cus * cfg.phase_a_blocks_per_cu);
    for (int k = 0; k < levels; ++k) {
        const int p = (k - 1) & 1, q = k & 1;
        uint64_t *lb_cur = v.lbstate + (size_t)q * v.lb_stride;
        uint64_t *lb_next = v.lbstate + (size_t)(q ^ 1) * v.lb_stride;
        if (k == 0) {
            hipLaunchKernelGGL(k_split<M>, dim3(nbs), dim3(kThreads), 0, s, v.recs, v.runstart,
                               v.dom_in_s, N, 0, v.fk[0], v.uk[0], v.urun[0], v.ucnt[0], v.rank_s,
                               v.fsize, v.usize, lb_cur, lb_next, v.sc);
        } else {
            hipLaunchKernelGGL(k_split<M>, dim3(nbs), dim3(kThreads), 0, s, v.uk[p], v.urun[p],
                               v.ucnt[p], -1, k, v.fk[q], v.uk[q], v.urun[q], v.ucnt[q], v.rank_s,
                               v.fsize, v.usize, lb_cur, lb_next, v.sc);
        }
        if (cfg.bitsets) {
            const int32_t fe = k < kProfLevels ? cfg.fprev[k] : 0;
            run_bit_level(v, v.fk[q], v.uk[q], v.urun[q], v.ucnt[q], k, ga, fe,
                          fe > 0 && fe <= cfg.lds_build_max, s);
        } else {
            hipLaunchKernelGGL(k_phase_a<M>, dim3(ga), dim3(kThreads), 0, s, v.fk[q], v.uk[q],
                               v.urun[q], v.ucnt[q], k, v.fsize, v.usize, v.work, v.sc);
        }
    }
    int32_t k0 = levels;
    uint32_t *fk0 = v.fk[0], *fk1 = v.fk[1], *uk0 = v.uk[0], *uk1 = v.uk[1];
    int32_t *urun0 = v.urun[0], *urun1 = v.urun[1], *ucnt0 = v.ucnt[0], *ucnt1 = v.ucnt[1];
    int32_t *rank_s = v.rank_s, *fsize = v.fsize, *usize = v.usize;
    uint32_t *blkcnt = v.blkcnt;
    DevScalars *sc = v.sc;
    GridBar *bar = v.bar;
    void *args[] = {&k0, &fk0, &fk1, &uk0, &uk1, &urun0, &urun1, &ucnt0, &ucnt1, &rank_s,
                    &fsize, &usize, &blkcnt, &sc, &bar};
    if (cfg.tail_block) {
        hipLaunchKernelGGL(k_peel_tail_block<M>, dim3(1), dim3(kThreads), 0, s, k0, fk0, fk1, uk0,
                           uk1, urun0, urun1, ucnt0, ucnt1, rank_s, fsize, usize, sc);
    } else {
        const int grid = cfg.num_cus * cfg.peel_blocks_per_cu;
        hipError_t e = hipLaunchCooperativeKernel((const void *)k_peel_tail<M>, dim3(grid),
                                                  dim3(kThreads), args, 0, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_last_front, dim3(1), dim3(64), 0, s, v.fsize, v.usize, v.N, v.K, v.sc);
    return hipGetLastError();
}

hipError_t run_peel(const SortViews &v, const LaunchCfg &cfg, hipStream_t s) {
    switch (v.M) {
#define NSGA3_CASE(m) case m: return launch_peel<m>(v, cfg, s);
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
}

int peel_max_blocks_per_cu(int M) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (M) {
#define NSGA3_OCC(m) case m: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_peel_tail<m>, kThreads, 0); break;
        NSGA3_OCC(2) NSGA3_OCC(3) NSGA3_OCC(4) NSGA3_OCC(5) NSGA3_OCC(6) NSGA3_OCC(7) NSGA3_OCC(8)
        NSGA3_OCC(9) NSGA3_OCC(10) NSGA3_OCC(11) NSGA3_OCC(12) NSGA3_OCC(13) NSGA3_OCC(14)
        NSGA3_OCC(15) NSGA3_OCC(16)
#undef NSGA3_OCC
        default: return 0;
    }
    return e == hipSuccess ? nb : 0;
}

size_t split_state_entries(int64_t N) { return (size_t)((N + kSplitTile - 1) / kSplitTile) + 1; }

}  // namespace nsga3
