// Nondominated sorting on gfx950: prepare order keys, presort by the exact key
// sum and count dominance over every unordered pair once (block bitsets, in
// bitdom.hip); the fronts are then peeled level by level (peel.hip), one split
// and one probe launch per level, with a one-work-group tail for the last ones.
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
#include "tile.h"

namespace nsga3 {

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
                                                         int32_t *__restrict__ runend,
                                                         const DevScalars *__restrict__ sc) {
    if (sc->err) return;
    const int MP = rec_stride(M);
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    const uint32_t i = sval[p];
    // the record in 16-byte stores (MP is a multiple of 4): whole lines reach
    // the L2 instead of one dword per lane 32 bytes apart
    uint4 *dst = reinterpret_cast<uint4 *>(recs + p * MP);
    for (int q = 0; q < MP / 4; ++q) {
        uint32_t v[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 4 * q + t;
            v[t] = k < M ? order_key(objs[(int64_t)i * M + k]) : (k == M ? (uint32_t)p : 0u);
        }
        dst[q] = make_uint4(v[0], v[1], v[2], v[3]);
    }
    // run bounds: most key sums are unique, so the neighbours usually settle
    // them; a binary search only inside a run of equal sums
    const uint64_t me = skey[p];
    int64_t lo = p, hi;
    if (p > 0 && skey[p - 1] == me) {
        lo = 0;  // first q in [0, p] with skey[q] == me
        hi = p;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skey[mid] < me) lo = mid + 1; else hi = mid;
        }
    }
    runstart[p] = (int32_t)lo;
    lo = p + 1;  // first q > p with a larger key sum
    if (p + 1 < N && skey[p + 1] == me) {
        hi = N;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if (skey[mid] <= me) lo = mid + 1; else hi = mid;
        }
    }
    runend[p] = (int32_t)lo;
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
    if (cfg.bitsets) {
        hipError_t e = run_bit_counts(v, s);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_domcount<M>, dim3((unsigned)items), dim3(kThreads), 0, s, v.recs,
                           v.runstart, (int32_t)N, v.dom_in_s, v.dom_out_s, v.sc);
    }
    v.mark();
    hipError_t e = run_peel(v, cfg, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scatter_orig, dim3((unsigned)((N + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, s, v.N, sval, v.rank_s, v.dom_in_s, v.dom_out_s, v.rank, v.dom_in,
                       v.dom_out, v.sc);
    return hipGetLastError();
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
                       v.recs, v.runstart, v.runend, v.sc);
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
