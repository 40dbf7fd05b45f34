// Nondominated sorting on gfx950: prepare order keys, presort by the exact key
// sum, count dominance over every unordered pair once, then peel the fronts in
// one persistent cooperative kernel.
//
// Pareto dominance follows Listing 1 / Eq. (6) (minimisation): i dominates j
// iff f_i <= f_j in every objective and f_i != f_j.  The dominance count of
// Eq. (7) is computed as the in-degree (number of dominators) of every point,
// which is what the front test p = 1{c = 0} of Eq. (8) / Alg. S.3 needs; the
// out-degree is returned beside it.  Fronts are peeled as in Eq. (9):
// c <- c - sum_i p_i D_ij for the points of the current front.
//
// Presort.  Every objective value is mapped to an order-preserving uint32 key
// (-0 and +0 share a key).  If i dominates j then key_i <= key_j in every
// objective with at least one strict inequality, so the 64-bit sum of the keys
// is strictly smaller for i.  Sorting by that sum is therefore a linear
// extension of dominance: only an earlier point can dominate a later one, and
// points with equal sums (in particular identical rows) never dominate each
// other.  Each unordered pair is decided by M unsigned compares
// ("all keys of the earlier point <= keys of the later point") instead of 2M.
#include "kernels.h"
#include "prims.h"

namespace nsga3 {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / kWave;
constexpr int kT = 4;                     // j points per lane
constexpr int kJT = kThreads * kT;        // j points per tile (block)
constexpr int kIC = kJT;                  // i points per chunk (dominance count)

// ---------------------------------------------------------------------------
// a0: order keys, key sums, ideal point (minimum key per objective), finiteness
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_prep(const float *__restrict__ objs, int64_t N, int M,
                                                   uint64_t *__restrict__ skey,
                                                   uint32_t *__restrict__ sval,
                                                   DevScalars *__restrict__ sc) {
    __shared__ uint32_t smin[16];
    if (threadIdx.x < 16) smin[threadIdx.x] = 0xffffffffu;
    __syncthreads();
    uint32_t lmin[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) lmin[k] = 0xffffffffu;
    bool bad = false;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        uint64_t s = 0;
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            if (k < M) {
                const float f = objs[i * M + k];
                bad |= !__builtin_isfinite(f);
                const uint32_t key = order_key(f);
                s += key;
                lmin[k] = key < lmin[k] ? key : lmin[k];
            }
        }
        skey[i] = s;
        sval[i] = (uint32_t)i;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        if (k < M) {
            const uint32_t v = wave_min(lmin[k]);
            if (lane_id() == 0) atomicMin(&smin[k], v);
        }
    }
    if (ballot(bad) && lane_id() == 0) atomicOr(&sc->err, (uint32_t)kErrNonfiniteObj);
    __syncthreads();
    if ((int)threadIdx.x < M) atomicMin(&sc->min_key[threadIdx.x], smin[threadIdx.x]);
}

// Sorted records: M keys, the sorted position, zero padding; and run starts
// (first sorted position with the same key sum).
__global__ __launch_bounds__(kThreads) void k_build_recs(const float *__restrict__ objs, int64_t N,
                                                         int M, const uint64_t *__restrict__ skey,
                                                         const uint32_t *__restrict__ sval,
                                                         uint32_t *__restrict__ recs,
                                                         int32_t *__restrict__ runstart,
                                                         const DevScalars *__restrict__ sc) {
    if (sc->err) return;
    const int MP = rec_stride(M);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const uint32_t i = sval[p];
    for (int k = 0; k < MP; ++k) {
        uint32_t v = 0;
        if (k < M) v = order_key(objs[(int64_t)i * M + k]);
        else if (k == M) v = (uint32_t)p;
        recs[p * MP + k] = v;
    }
    const uint64_t me = skey[p];
    int64_t lo = 0, hi = p;  // first q in [0, p] with skey[q] == me
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (skey[mid] < me) lo = mid + 1; else hi = mid;
    }
    runstart[p] = (int32_t)lo;
}

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
// points.  Records are fetched in groups of kU so the scalar loads overlap.
// With kCountOut, lane 0 stores the per-record counts to out_row[0..n).
template <int M, bool kChecked, bool kCountOut>
__device__ __forceinline__ void tile_rows(const uint32_t *__restrict__ rec, int n,
                                          const uint32_t (&kj)[kT][M], const int32_t (&run)[kT],
                                          int32_t (&cin)[kT], uint32_t *__restrict__ out_row,
                                          bool lane0) {
    constexpr int kU = 4;
    constexpr int MP = rec_stride(M);
    int ii = 0;
    for (; ii + kU <= n; ii += kU) {
        uint32_t ki[kU][M];
        int ipos[kU];
        const uint32_t *g = rec + (size_t)ii * MP;  // one base, constant offsets
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
        const uint32_t *r = rec + (size_t)ii * MP;
        uint32_t ki[M];
#pragma unroll
        for (int k = 0; k < M; ++k) ki[k] = r[k];
        const int ipos = kChecked ? (int)r[M] : 0;
        const uint32_t c = tile_one<M, kChecked, kCountOut>(ki, ipos, kj, run, cin);
        if (kCountOut && lane0) out_row[ii] = c;
    }
}

// ---------------------------------------------------------------------------
// a1: dominance counts over the upper triangle of (i-chunk, j-tile) pairs.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kThreads) void k_domcount(const uint32_t *__restrict__ recs,
                                                       const int32_t *__restrict__ runstart,
                                                       int32_t N, int32_t *__restrict__ dom_in,
                                                       int32_t *__restrict__ dom_out,
                                                       const DevScalars *__restrict__ sc) {
    constexpr int MP = rec_stride(M);
    __shared__ uint32_t obuf[kWaves][kIC];
    if (sc->err) return;
    const uint32_t b = blockIdx.x;
    uint32_t jt = (uint32_t)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
    while ((uint64_t)(jt + 1) * (jt + 2) / 2 <= b) ++jt;
    while ((uint64_t)jt * (jt + 1) / 2 > b) --jt;
    const uint32_t ic = b - jt * (jt + 1) / 2;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    const int lane = (int)lane_id();
    const int i0 = (int)ic * kIC;
    const int jbase = (int)jt * kJT + w * kWave * kT;

    for (int x = lane; x < kIC; x += kWave) obuf[w][x] = 0;

    uint32_t kj[kT][M];
    int32_t run[kT], cin[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int q = jbase + t * kWave + lane;
        cin[t] = 0;
        if (q < N) {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = recs[(size_t)q * MP + k];
            run[t] = runstart[q];
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = 0u;  // below every finite key: never dominated
            run[t] = 0;
        }
    }
    if (jbase < N) {
        const int qlast = min(jbase + kWave * kT - 1, N - 1);
        const int run_lo = runstart[jbase];
        const int run_hi = runstart[qlast];
        const int iend = min(i0 + kIC, run_hi);
        const int ifast = min(max(run_lo, i0), iend);
        const bool lane0 = lane == 0;
        if (ifast > i0)
            tile_rows<M, false, true>(recs + (size_t)i0 * MP, ifast - i0, kj, run, cin,
                                      &obuf[w][0], lane0);
        if (iend > ifast)
            tile_rows<M, true, true>(recs + (size_t)ifast * MP, iend - ifast, kj, run, cin,
                                     &obuf[w][ifast - i0], lane0);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int q = jbase + t * kWave + lane;
        if (q < N && cin[t]) atomicAdd(&dom_in[q], cin[t]);
    }
    if (dom_out) {
        for (int x = threadIdx.x; x < kIC; x += kThreads) {
            uint32_t s = 0;
#pragma unroll
            for (int q = 0; q < kWaves; ++q) s += obuf[q][x];
            if (s && i0 + x < N) atomicAdd(&dom_out[i0 + x], (int32_t)s);
        }
    }
}

// ---------------------------------------------------------------------------
// a2/a3: persistent front peeling (cooperative launch, grid barriers).
//
// Lists kept in sorted-position order, double buffered across levels:
//   F (current front): records (keys + position)
//   U (unranked):      records, run starts, remaining in-degree
// Level k: every U point subtracts the number of its dominators in F_k
// (phase A), then U is split into F_{k+1} (count reached zero) and U_{k+1}.
// ---------------------------------------------------------------------------
struct PeelPtrs {
    uint32_t *fk0, *fk1, *uk0, *uk1;
    int32_t *urun0, *urun1, *ucnt0, *ucnt1;
};

// Split the list src (n records, sorted by position) into the points whose
// remaining in-degree is zero -- the next front, appended to fdst with rank
// `level` -- and the rest, appended to udst; both keep sorted order.
// Returns false when a barrier failed.
template <int M>
__device__ bool classify(const uint32_t *__restrict__ srec, const int32_t *__restrict__ srun,
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
    // prefix over earlier blocks and totals
    uint32_t pf = 0, pu = 0, tf = 0, tu = 0;
    for (uint32_t q = threadIdx.x; q < G; q += kThreads) {
        const uint32_t a = __hip_atomic_load(&blkcnt[2 * q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t c = __hip_atomic_load(&blkcnt[2 * q + 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tf += a; tu += c;
        if (q < blockIdx.x) { pf += a; pu += c; }
    }
    pf = wave_sum(pf); pu = wave_sum(pu); tf = wave_sum(tf); tu = wave_sum(tu);
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
    // ordered write
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
            const uint4 *r = reinterpret_cast<const uint4 *>(srec + (size_t)e * MP);
            uint4 v[MP / 4];
#pragma unroll
            for (int k = 0; k < MP / 4; ++k) v[k] = r[k];
            const uint32_t pos = srec[(size_t)e * MP + M];
            if (isf) {
                uint4 *d = reinterpret_cast<uint4 *>(fdst + (size_t)(pf + exf) * MP);
#pragma unroll
                for (int k = 0; k < MP / 4; ++k) d[k] = v[k];
                rank_s[pos] = level;
            } else {
                const uint32_t slot = pu + exu;
                uint4 *d = reinterpret_cast<uint4 *>(udst + (size_t)slot * MP);
#pragma unroll
                for (int k = 0; k < MP / 4; ++k) d[k] = v[k];
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

// Front members staged in LDS per work item: 32 KiB of records.
template <int M>
struct PeelTile {
    static constexpr int MP = rec_stride(M);
    static constexpr int IC = 8192 / MP;  // records per chunk
};

// Smallest index in [lo, hi) of the LDS-staged chunk whose position is >= bound.
template <int M>
__device__ __forceinline__ int lds_lower_bound(const uint32_t *lrec, int lo, int hi, int bound) {
    constexpr int MP = rec_stride(M);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((int)lrec[mid * MP + M] < bound) lo = mid + 1; else hi = mid;
    }
    return lo;
}

template <int M>
__device__ void peel_phase_a(const uint32_t *__restrict__ fk, int32_t nf,
                             const uint32_t *__restrict__ uk, const int32_t *__restrict__ urun,
                             int32_t *__restrict__ ucnt, int32_t nu, uint32_t *lrec) {
    constexpr int MP = rec_stride(M);
    constexpr int IC = PeelTile<M>::IC;
    const int nIC = (nf + IC - 1) / IC;
    const int nJT = (nu + kJT - 1) / kJT;
    const int64_t nitems = (int64_t)nIC * nJT;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    for (int64_t item = blockIdx.x; item < nitems; item += gridDim.x) {
        const int jt = (int)(item % nJT);
        const int ic = (int)(item / nJT);
        const int f0 = ic * IC;
        const int f1 = min(f0 + IC, nf);
        const int tile_last = min(jt * kJT + kJT - 1, nu - 1);
        if ((int)fk[(size_t)f0 * MP + M] >= urun[tile_last]) continue;  // block-uniform skip
        __syncthreads();  // previous item's readers are done with lrec
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
            const int n = f1 - f0;
            const int iend = lds_lower_bound<M>(lrec, 0, n, run_hi);
            const int ifast = lds_lower_bound<M>(lrec, 0, iend, run_lo);
            if (ifast > 0)
                tile_rows<M, false, false>(lrec, ifast, kj, run, cin, nullptr, false);
            if (iend > ifast)
                tile_rows<M, true, false>(lrec + (size_t)ifast * MP, iend - ifast, kj, run, cin,
                                          nullptr, false);
#pragma unroll
            for (int t = 0; t < kT; ++t) {
                const int q = jbase + t * kWave + lane;
                if (q < nu && cin[t]) atomicSub(&ucnt[q], cin[t]);
            }
        }
    }
}

template <int M>
__global__ __launch_bounds__(kThreads) void k_peel(
    const uint32_t *__restrict__ recs, const int32_t *__restrict__ runstart,
    const int32_t *__restrict__ dom_in_s, int32_t N, int64_t K, uint32_t *__restrict__ fk0,
    uint32_t *__restrict__ fk1, uint32_t *__restrict__ uk0, uint32_t *__restrict__ uk1,
    int32_t *__restrict__ urun0, int32_t *__restrict__ urun1, int32_t *__restrict__ ucnt0,
    int32_t *__restrict__ ucnt1, int32_t *__restrict__ rank_s, int32_t *__restrict__ fsize,
    uint32_t *__restrict__ blkcnt, DevScalars *__restrict__ sc, GridBar *__restrict__ bar) {
    __shared__ __attribute__((aligned(16))) uint32_t lrec[8192];
    if (__hip_atomic_load(&sc->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) return;
    int32_t nf = 0, nu = 0;
    // level 0: split all points by their dominance count
    if (!classify<M>(recs, runstart, dom_in_s, N, fk0, uk0, urun0, ucnt0, rank_s, 0, blkcnt, sc, bar,
                     &nf, &nu))
        return;
    if (blockIdx.x == 0 && threadIdx.x == 0) fsize[0] = nf;
    int cur = 0;
    int32_t level = 0;
    bool ok = grid_barrier2(bar, &sc->err);
    while (ok && nu > 0) {
        if (nf == 0) {  // impossible for a partial order; leave instead of spinning
            if (blockIdx.x == 0 && threadIdx.x == 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
            break;
        }
        uint32_t *fc = cur ? fk1 : fk0, *fn = cur ? fk0 : fk1;
        uint32_t *uc = cur ? uk1 : uk0, *un = cur ? uk0 : uk1;
        int32_t *rc = cur ? urun1 : urun0, *rn = cur ? urun0 : urun1;
        int32_t *cc = cur ? ucnt1 : ucnt0, *cn = cur ? ucnt0 : ucnt1;
        peel_phase_a<M>(fc, nf, uc, rc, cc, nu, lrec);
        if (!grid_barrier2(bar, &sc->err)) { ok = false; break; }
        int32_t nf2 = 0, nu2 = 0;
        if (!classify<M>(uc, rc, cc, nu, fn, un, rn, cn, rank_s, level + 1, blkcnt, sc, bar, &nf2,
                         &nu2)) {
            ok = false;
            break;
        }
        ++level;
        if (blockIdx.x == 0 && threadIdx.x == 0) fsize[level] = nf2;
        nf = nf2;
        nu = nu2;
        cur ^= 1;
        ok = grid_barrier2(bar, &sc->err);
    }
    if (ok && blockIdx.x == 0 && threadIdx.x == 0) {
        // a3: l = rank of the K-th smallest rank (0-based position K-1)
        const int32_t L = level + 1;
        int64_t cum = 0;
        int32_t l = L - 1;
        for (int32_t k = 0; k < L; ++k) {
            const int64_t sz = __hip_atomic_load(&fsize[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (cum + sz >= K) { l = k; break; }
            cum += sz;
        }
        const int64_t szl = __hip_atomic_load(&fsize[l], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        sc->num_fronts = L;
        sc->last_front = l;
        sc->last_front_size = (int32_t)szl;
        sc->n_before = cum;
        sc->num_from_last = K - cum;
    }
}

// Original-order outputs of the sorting stage.
__global__ __launch_bounds__(kThreads) void k_scatter_orig(int64_t N, const uint32_t *__restrict__ sval,
                                                           const int32_t *__restrict__ rank_s,
                                                           const int32_t *__restrict__ din_s,
                                                           const int32_t *__restrict__ dout_s,
                                                           int32_t *__restrict__ rank,
                                                           int32_t *__restrict__ din,
                                                           int32_t *__restrict__ dout,
                                                           const DevScalars *__restrict__ sc) {
    if (sc->err) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const uint32_t i = sval[p];
    rank[i] = rank_s[p];
    if (din) din[i] = din_s[p];
    if (dout) dout[i] = dout_s[p];
}

template <int M>
static hipError_t launch_counts_and_peel(const SortViews &v, const uint32_t *sval,
                                         const LaunchCfg &cfg, hipStream_t s) {
    const int N = (int)v.N;
    const int64_t nJT = (N + kJT - 1) / kJT;
    const int64_t items = nJT * (nJT + 1) / 2;
    v.mark();
    hipLaunchKernelGGL(k_domcount<M>, dim3((unsigned)items), dim3(kThreads), 0, s, v.recs,
                       v.runstart, (int32_t)N, v.dom_in_s, v.dom_out_s, v.sc);
    v.mark();
    const uint32_t *recs = v.recs;
    const int32_t *runstart = v.runstart;
    const int32_t *dom_in_s = v.dom_in_s;
    int32_t n32 = N;
    int64_t K = v.K;
    uint32_t *fk0 = v.fk[0], *fk1 = v.fk[1], *uk0 = v.uk[0], *uk1 = v.uk[1];
    int32_t *urun0 = v.urun[0], *urun1 = v.urun[1], *ucnt0 = v.ucnt[0], *ucnt1 = v.ucnt[1];
    int32_t *rank_s = v.rank_s, *fsize = v.fsize;
    uint32_t *blkcnt = v.blkcnt;
    DevScalars *sc = v.sc;
    GridBar *bar = v.bar;
    void *args[] = {&recs, &runstart, &dom_in_s, &n32, &K, &fk0, &fk1, &uk0, &uk1, &urun0,
                    &urun1, &ucnt0, &ucnt1, &rank_s, &fsize, &blkcnt, &sc, &bar};
    const int grid = cfg.num_cus * cfg.peel_blocks_per_cu;
    hipError_t e = hipLaunchCooperativeKernel((const void *)k_peel<M>, dim3(grid), dim3(kThreads),
                                              args, 0, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_orig, dim3((unsigned)((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, s, v.N, sval, v.rank_s, v.dom_in_s, v.dom_out_s, v.rank, v.dom_in,
                       v.dom_out, v.sc);
    return hipGetLastError();
}

int peel_max_blocks_per_cu(int M) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (M) {
#define NSGA3_OCC(m) case m: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_peel<m>, kThreads, 0); break;
        NSGA3_OCC(2) NSGA3_OCC(3) NSGA3_OCC(4) NSGA3_OCC(5) NSGA3_OCC(6) NSGA3_OCC(7) NSGA3_OCC(8)
        NSGA3_OCC(9) NSGA3_OCC(10) NSGA3_OCC(11) NSGA3_OCC(12) NSGA3_OCC(13) NSGA3_OCC(14)
        NSGA3_OCC(15) NSGA3_OCC(16)
#undef NSGA3_OCC
        default: return 0;
    }
    return e == hipSuccess ? nb : 0;
}

hipError_t run_sort_stage(const SortViews &v, const LaunchCfg &cfg, hipStream_t s) {
    const int64_t N = v.N;
    const unsigned nbN = (unsigned)((N + kThreads - 1) / kThreads);
    const unsigned nbPrep = nbN < 2048u ? nbN : 2048u;
    hipLaunchKernelGGL(k_prep, dim3(nbPrep), dim3(kThreads), 0, s, v.objs, N, v.M, v.skey, v.sval, v.sc);
    // key sums need at most 32 + 4 bits for M <= 16
    bool in_alt = false;
    radix_sort_pairs(v.skey, v.sval, v.skey_alt, v.sval_alt, N, 40, v.temp, s, &in_alt);
    const uint64_t *skey = in_alt ? v.skey_alt : v.skey;
    const uint32_t *sval = in_alt ? v.sval_alt : v.sval;
    hipLaunchKernelGGL(k_build_recs, dim3(nbN), dim3(kThreads), 0, s, v.objs, N, v.M, skey, sval,
                       v.recs, v.runstart, v.sc);
    switch (v.M) {
#define NSGA3_CASE(m) case m: return launch_counts_and_peel<m>(v, sval, cfg, s);
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace nsga3
