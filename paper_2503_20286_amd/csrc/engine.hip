// Batched selection engine: one persistent kernel per objective count runs
// many independent environmental selections (Alg. S.4 with the sorting of
// Alg. S.3 and the niching of Alg. S.1) as work items.
//
// Each instance walks through the stages of engine.h.  A worker block claims
// one item of any instance whose current stage has unclaimed items (one
// 64-bit atomic add on the instance's progress word), runs it, and counts it
// done; the block that finishes the last item of a stage runs that stage's
// short epilogue (scans, the intercept solve, the niching threshold) and
// publishes the next stage.  Items never wait for other items, so any number
// of resident blocks makes progress, and blocks leave when every instance of
// the launch is done (or after a long idle period, flagged as an error).
//
// Memory ordering: every wave of a finishing block waits for its stores to
// reach the L2, then one agent-scope release fence writes them back before the
// block counts its item; the epilogue block
// acquires before reading, and publishes the next stage with a release
// store; claimers acquire after a successful claim.  Data written inside the
// kernel is never read through the scalar cache (which vector stores do not
// update): uniform reads of such data use relaxed atomic loads, and record
// lists are staged through LDS with vector loads.
//
// The per-item arithmetic is the single-selection arithmetic (same key map,
// same presort, same float64 solve and re-scoring), so every output is
// identical to a single nsga3_select call on the same instance.
#include <float.h>

#include "bitdom.h"
#include "engine.h"
#include "prims.h"
#include "stage_math.h"
#include "tile.h"

namespace nsga3 {

namespace {

constexpr unsigned long long kIdleLimit = 400000000ull;  // wall-clock ticks (seconds at 100 MHz)

// Uniform reads of data written inside the kernel.  A workgroup-scope atomic
// load is a vector load that may hit the caches (which the claim's acquire
// made current) but is never served by the scalar cache.
template <typename T>
__device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ double ldd(const double *p) {
    return __builtin_bit_cast(double, ld(reinterpret_cast<const uint64_t *>(p)));
}

// Reads of words other blocks update concurrently (progress words, counters).
template <typename T>
__device__ __forceinline__ T lda(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ T *at(char *w, size_t off) {
    return reinterpret_cast<T *>(w + off);
}

template <int MP>
__device__ __forceinline__ void copy_rec(uint32_t *d, const uint32_t *s) {
#pragma unroll
    for (int k = 0; k < MP / 4; ++k)
        reinterpret_cast<uint4 *>(d)[k] = reinterpret_cast<const uint4 *>(s)[k];
}

// Dword c of a 16-byte vector.
template <int c>
__device__ __forceinline__ uint32_t vec_dword(const uint4 &v) {
    if constexpr (c == 0) return v.x;
    else if constexpr (c == 1) return v.y;
    else if constexpr (c == 2) return v.z;
    else return v.w;
}

// Cooperative copy of n records (MP dwords each) into LDS.
template <int MP>
__device__ __forceinline__ void stage_recs(uint32_t *lds, const uint32_t *src, int32_t n) {
    const uint4 *s = reinterpret_cast<const uint4 *>(src);
    uint4 *d = reinterpret_cast<uint4 *>(lds);
    const int32_t nvec = n * (MP / 4);
    for (int32_t q = threadIdx.x; q < nvec; q += kEThreads) d[q] = s[q];
}

// ---------------------------------------------------------------------------
// Items
// ---------------------------------------------------------------------------

// a0: keys, key sums, ideal point, finiteness (first cdiv(N, kEChunk) items);
// unit references and zeroed niche counters (remaining items).
template <int M>
__device__ void item_prep(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t N = I.N;
    const int32_t C1 = (int32_t)cdiv(N, kEChunk);
    if (t >= C1) {
        const int32_t j = (t - C1) * kEThreads + (int32_t)threadIdx.x;
        if (j < I.H) {
            at<int32_t>(w, L.rho)[j] = 0;
            at<int32_t>(w, L.bcount)[j] = 0;
            if (!unit_reference(I.refs, j, M, at<double>(w, L.rhat64), at<float>(w, L.rhat32)))
                atomicOr(&sc->err, (uint32_t)kErrBadRef);
        }
        return;
    }
    uint32_t *smin = smem;
    if (threadIdx.x < M) smin[threadIdx.x] = 0xffffffffu;
    __syncthreads();
    uint32_t lmin[M];
#pragma unroll
    for (int k = 0; k < M; ++k) lmin[k] = 0xffffffffu;
    unsigned long long smn = ~0ull, smx = 0ull;  // range of the sum keys
    bool bad = false;
    uint64_t *skey = at<uint64_t>(w, L.skey0);
    uint32_t *sval = at<uint32_t>(w, L.sval0);
    int32_t *din = at<int32_t>(w, L.din), *dout = at<int32_t>(w, L.dout);
    for (int q = 0; q < kEChunk / kEThreads; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        if (p < N) {
            uint64_t s = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const float f = I.objs[(int64_t)p * M + k];
                bad |= !__builtin_isfinite(f);
                const uint32_t key = order_key(f);
                s += key;
                lmin[k] = key < lmin[k] ? key : lmin[k];
            }
            if (M == 2) {  // lexicographic pair (see radix_passes)
                const uint32_t k0 = order_key(I.objs[(int64_t)p * M]);
                const uint32_t k1 = order_key(I.objs[(int64_t)p * M + 1]);
                s = ((uint64_t)k0 << 32) | (uint64_t)k1;
            } else {
                smn = s < smn ? s : smn;
                smx = s > smx ? s : smx;
            }
            skey[p] = s;
            sval[p] = (uint32_t)p;
            din[p] = 0;
            dout[p] = 0;
        }
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint32_t v = wave_min(lmin[k]);
        if (lane_id() == 0) atomicMin(&smin[k], v);
    }
    if (ballot(bad) && lane_id() == 0) atomicOr(&sc->err, (uint32_t)kErrNonfiniteObj);
    if (M != 2) {
        smn = wave_min(smn);
        smx = wave_max(smx);
        if (lane_id() == 0 && smn <= smx) {
            atomicMin(&sc->skey_min, smn);
            atomicMax(&sc->skey_max, smx);
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < M) atomicMin(&sc->min_key[threadIdx.x], smin[threadIdx.x]);
}

// What the radix passes subtract from the presort keys: the smallest sum key
// (M >= 3), so that the passes cover only the instance's key range.
__device__ __forceinline__ uint64_t key_base(const EInst &I, char *w) {
    return I.M == 2 ? 0ull : ld(&at<EScal>(w, I.L.scal)->skey_min);
}

// Presort passes of an instance (set by the key-and-reference epilogue).
__device__ __forceinline__ int sort_passes(const EInst &I) {
    return ld(&at<EScal>(I.ws, I.L.scal)->rs_passes);
}

// Radix histogram of one tile (block-major: hist[tile][digit]).
__device__ void item_hist(const EInst &I, int pass, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const uint64_t *keys = at<uint64_t>(w, (pass & 1) ? L.skey1 : L.skey0);
    const uint64_t kmin = key_base(I, w);
    uint32_t *h = smem;
    h[threadIdx.x] = 0;
    __syncthreads();
    const int shift = 8 * pass;
#pragma unroll
    for (int it = 0; it < kERsTile / kEThreads; ++it) {
        const int32_t p = t * kERsTile + it * kEThreads + (int32_t)threadIdx.x;
        if (p < I.N) atomicAdd(&h[(uint32_t)((keys[p] - kmin) >> shift) & 255u], 1u);
    }
    __syncthreads();
    at<uint32_t>(w, L.hist)[(size_t)t * 256 + threadIdx.x] = h[threadIdx.x];
}

// Stable radix scatter of one tile; the tile's digit offsets are summed from
// the histogram (all keys with a smaller digit, plus equal digits in earlier
// tiles).
__device__ void item_scat(const EInst &I, int pass, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const int32_t N = I.N;
    const int32_t nt = (int32_t)cdiv(N, kERsTile);
    const uint64_t *kin = at<uint64_t>(w, (pass & 1) ? L.skey1 : L.skey0);
    const uint32_t *vin = at<uint32_t>(w, (pass & 1) ? L.sval1 : L.sval0);
    uint64_t *kout = at<uint64_t>(w, (pass & 1) ? L.skey0 : L.skey1);
    uint32_t *vout = at<uint32_t>(w, (pass & 1) ? L.sval0 : L.sval1);
    const uint32_t *hist = at<uint32_t>(w, L.hist);
    uint32_t *base_off = smem;
    uint32_t *run = smem + 256;
    uint32_t *wc = smem + 512;          // [kEThreads / 64][256]
    uint32_t *scan_lds = smem + 512 + 4 * 256;
    const uint32_t tid = threadIdx.x;
    const uint32_t wv = tid / kWave;
    {
        uint32_t before = 0, total = 0;
        for (int32_t b = 0; b < nt; ++b) {
            const uint32_t h = hist[(size_t)b * 256 + tid];
            total += h;
            before += b < t ? h : 0u;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(total, scan_lds, &tot);
        base_off[tid] = ex + before;
        run[tid] = 0;
    }
    __syncthreads();
    const int shift = 8 * pass;
    const uint64_t kmin = key_base(I, w);
    for (int it = 0; it < kERsTile / kEThreads; ++it) {
#pragma unroll
        for (int q = 0; q < kEThreads / kWave; ++q) wc[q * 256 + tid] = 0;
        __syncthreads();
        const int32_t p = t * kERsTile + it * kEThreads + (int32_t)tid;
        const bool valid = p < N;
        const uint64_t key = valid ? kin[p] : 0ull;
        const uint32_t d = (uint32_t)((key - kmin) >> shift) & 255u;
        uint64_t m = ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t below = lanes_below(m);
        const uint32_t cnt = (uint32_t)__popcll(m);
        if (valid && below == cnt - 1) wc[wv * 256 + d] = cnt;
        __syncthreads();
        if (valid) {
            uint32_t pre = run[d];
            for (uint32_t q = 0; q < wv; ++q) pre += wc[q * 256 + d];
            const uint32_t dst = base_off[d] + pre + below;
            kout[dst] = key;
            vout[dst] = vin[p];
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int q = 0; q < kEThreads / kWave; ++q) add += wc[q * 256 + tid];
        run[tid] += add;
        __syncthreads();
    }
}

// Sorted records (M keys, position, padding) and run starts and ends (runs
// of equal sort keys).  A thread's loads (positions, sort keys and their
// neighbours, then the objective values) are issued before its stores; a run
// bound is searched for only when a neighbour has the same key (otherwise it
// is the point itself), as in the single-selection records kernel.  On the
// 512-instance batch this took the stage from 328 to 314 block-ms per launch
// (two binary searches per point before).
template <int M>
__device__ void item_recs(const EInst &I, int32_t t) {
    const ELayout &L = I.L;
    constexpr int MP = rec_stride(M);
    constexpr int kQ = kEChunk / kEThreads;
    char *w = I.ws;
    const int32_t N = I.N;
    const bool odd = (sort_passes(I) & 1) != 0;  // where the last pass wrote
    const uint64_t *skey = at<uint64_t>(w, odd ? L.skey1 : L.skey0);
    const uint32_t *sval = at<uint32_t>(w, odd ? L.sval1 : L.sval0);
    uint32_t *recs = at<uint32_t>(w, L.recs);
    int32_t *runstart = at<int32_t>(w, L.runstart);
    int32_t *runend = at<int32_t>(w, L.runend);
    uint32_t idx[kQ];
    uint64_t me[kQ];
    bool eq_prev[kQ], eq_next[kQ];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        idx[q] = 0;
        me[q] = 0;
        eq_prev[q] = eq_next[q] = false;
        if (p < N) {
            idx[q] = sval[p];
            me[q] = skey[p];
            eq_prev[q] = p > 0 && skey[p - 1] == me[q];
            eq_next[q] = p + 1 < N && skey[p + 1] == me[q];
        }
    }
    float f[kQ][M];
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
#pragma unroll
        for (int k = 0; k < M; ++k) f[q][k] = p < N ? I.objs[(int64_t)idx[q] * M + k] : 0.0f;
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        if (p >= N) break;
        uint32_t v[MP];
#pragma unroll
        for (int k = 0; k < MP; ++k)
            v[k] = k < M ? order_key(f[q][k]) : (k == M ? (uint32_t)p : 0u);
#pragma unroll
        for (int k = 0; k < MP / 4; ++k)
            reinterpret_cast<uint4 *>(recs + (size_t)p * MP)[k] =
                make_uint4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        if (p >= N) break;
        int32_t lo = p, hi = p;
        if (eq_prev[q]) {  // first position with this key
            lo = 0;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (skey[mid] < me[q]) lo = mid + 1; else hi = mid;
            }
        }
        runstart[p] = lo;
        lo = p + 1;  // first position with a larger key
        if (eq_next[q]) {
            hi = N;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                if (skey[mid] <= me[q]) lo = mid + 1; else hi = mid;
            }
        }
        runend[p] = lo;
    }
}

// a1: dominance counts of one (i-chunk, j-tile) pair of the triangle.  The
// records are written once per launch (before any item of this stage reads
// them), so the earlier points stream through the scalar cache as in the
// single-selection kernel.
typedef __attribute__((address_space(4))) const uint32_t const_u32;

template <int M>
__device__ void item_dom(const EInst &I, int32_t b, uint32_t *smem) {
    const ELayout &L = I.L;
    constexpr int MP = rec_stride(M);
    constexpr int IC = kJT;
    char *w = I.ws;
    const int32_t N = I.N;
    uint32_t jt = (uint32_t)((sqrtf(8.0f * (float)b + 1.0f) - 1.0f) * 0.5f);
    while ((uint64_t)(jt + 1) * (jt + 2) / 2 <= (uint32_t)b) ++jt;
    while ((uint64_t)jt * (jt + 1) / 2 > (uint32_t)b) --jt;
    const int32_t ic = b - (int32_t)(jt * (jt + 1) / 2);
    const int32_t i0 = ic * IC;
    const int32_t jt0 = (int32_t)jt * kJT;
    const uint32_t *recs = at<uint32_t>(w, L.recs);
    const const_u32 *srec = (const const_u32 *)recs;
    const int32_t *runstart = at<int32_t>(w, L.runstart);
    int32_t *din = at<int32_t>(w, L.din), *dout = at<int32_t>(w, L.dout);
    if (i0 >= N) return;
    uint32_t *obuf = smem;  // [kWaves][IC]
    for (int x = threadIdx.x; x < kWaves * IC; x += kEThreads) obuf[x] = 0;
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    const int32_t jbase = jt0 + wv * kWave * kT;
    uint32_t kj[kT][M];
    int32_t run[kT], cin[kT];
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int32_t q = jbase + t * kWave + lane;
        cin[t] = 0;
        if (q < N) {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = recs[(size_t)q * MP + k];
            run[t] = runstart[q];
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k) kj[t][k] = 0u;
            run[t] = 0;
        }
    }
    int32_t i1 = min(i0 + IC, N);
    if (jbase < N) {
        const int32_t qlast = min(jbase + kWave * kT - 1, N - 1);
        const int32_t run_lo = ld(&runstart[jbase]);
        const int32_t run_hi = ld(&runstart[qlast]);
        const int32_t iend = min(i1, run_hi);
        const int32_t ifast = min(max(run_lo, i0), iend);
        const bool lane0 = lane == 0;
        if (ifast > i0)
            tile_rows<M, false, true>(srec + (size_t)i0 * MP, ifast - i0, kj, run, cin,
                                      obuf + wv * IC, lane0);
        if (iend > ifast)
            tile_rows<M, true, true>(srec + (size_t)ifast * MP, iend - ifast, kj, run, cin,
                                     obuf + wv * IC + (ifast - i0), lane0);
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kT; ++t) {
        const int32_t q = jbase + t * kWave + lane;
        if (q < N && cin[t]) atomicAdd(&din[q], cin[t]);
    }
    for (int x = threadIdx.x; x < i1 - i0; x += kEThreads) {
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) s += obuf[q * IC + x];
        if (s) atomicAdd(&dout[i0 + x], (int32_t)s);
    }
}

// Level-k list sources: level 0 reads every sorted point; later levels read
// the previous level's remaining list.
struct LevelLists {
    const uint32_t *srec;
    const int32_t *srun, *scnt;
    uint32_t *fdst, *udst;
    int32_t *rdst, *cdst;
};

__device__ __forceinline__ LevelLists level_lists(char *w, const ELayout &L, int32_t k) {
    LevelLists s;
    const bool odd_prev = ((k - 1) & 1) != 0;
    if (k == 0) {
        s.srec = at<uint32_t>(w, L.recs);
        s.srun = at<int32_t>(w, L.runstart);
        s.scnt = at<int32_t>(w, L.din);
    } else {
        s.srec = at<uint32_t>(w, odd_prev ? L.uk1 : L.uk0);
        s.srun = at<int32_t>(w, odd_prev ? L.urun1 : L.urun0);
        s.scnt = at<int32_t>(w, odd_prev ? L.ucnt1 : L.ucnt0);
    }
    const bool odd = (k & 1) != 0;
    s.fdst = at<uint32_t>(w, odd ? L.fk1 : L.fk0);
    s.udst = at<uint32_t>(w, odd ? L.uk1 : L.uk0);
    s.rdst = at<int32_t>(w, odd ? L.urun1 : L.urun0);
    s.cdst = at<int32_t>(w, odd ? L.ucnt1 : L.ucnt0);
    return s;
}

// Split, counting pass: fronts (remaining in-degree 0) and the rest per item.
__device__ void item_splitc(const EInst &I, int32_t k, int32_t n, int32_t t,
                            uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const LevelLists s = level_lists(w, L, k);
    const int32_t s0 = t * kESplit, s1 = min(s0 + kESplit, n);
    uint32_t nz = 0, nn = 0;
    for (int32_t e = s0 + (int32_t)threadIdx.x; e < s1; e += kEThreads) {
        if (s.scnt[e] == 0) ++nz; else ++nn;
    }
    nz = wave_sum(nz);
    nn = wave_sum(nn);
    if (lane_id() == 0) {
        smem[threadIdx.x / kWave] = nz;
        smem[kWaves + threadIdx.x / kWave] = nn;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, c = 0;
        for (int q = 0; q < kWaves; ++q) { a += smem[q]; c += smem[kWaves + q]; }
        uint32_t *spc = at<uint32_t>(w, L.spc);
        spc[2 * t] = a;
        spc[2 * t + 1] = c;
    }
}

// Ordered split of list entries [e0, e1) (at most kESplit) into F_k (rank k)
// and U_k at output offsets (of, ou).  Entry e0 + q * kEThreads + t belongs
// to thread t, so every load and store instruction covers consecutive
// entries.  All loads of a thread (counts, run starts, records) are issued
// before its first store: the destination lists never overlap the source
// list, and a worker block has one wave per SIMD, so loads interleaved with
// the stores would cost a memory round trip each.  Offsets: a ballot per
// (q, wave) gives the fronts before an entry inside its wave; the waves'
// counts go through LDS once.  Returns the chunk's front and remaining counts.
// On the 512-instance batch (ms per launch), consecutive entries per thread
// and one packed block scan: 8 entries with loads and stores interleaved
// 11.1-11.2; with every load first, 16, 8, 4, 2 and 1 entries 11.7, 11.0,
// 10.7, 10.5 and 10.4; this form with 8, 2 or 1 entries 10.6, 10.4, 10.4.
template <int M>
__device__ void split_chunk(const LevelLists &s, int32_t k, int32_t e0, int32_t e1, uint32_t of,
                            uint32_t ou, int32_t *rank_s, uint32_t *lds, uint32_t *nf,
                            uint32_t *nu) {
    constexpr int MP = rec_stride(M);
    constexpr int MV = MP / 4;
    constexpr int kPer = kESplit / kEThreads;
    constexpr int kEW = kEThreads / kWave;
    const int lane = (int)lane_id();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    int32_t cnt[kPer], run[kPer];
    uint4 rec[kPer][MV];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int32_t e = e0 + q * kEThreads + (int32_t)threadIdx.x;
        if (e < e1) {
            cnt[q] = s.scnt[e];
            run[q] = s.srun[e];
            const uint4 *r = reinterpret_cast<const uint4 *>(s.srec + (size_t)e * MP);
#pragma unroll
            for (int v = 0; v < MV; ++v) rec[q][v] = r[v];
        } else {
            cnt[q] = -1;
            run[q] = 0;
#pragma unroll
            for (int v = 0; v < MV; ++v) rec[q][v] = make_uint4(0u, 0u, 0u, 0u);
        }
    }
    uint64_t fm[kPer];
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        fm[q] = ballot(cnt[q] == 0);
        if (lane == 0) lds[q * kEW + wv] = (uint32_t)__popcll(fm[q]);
    }
    __syncthreads();
    uint32_t before[kPer], tf = 0;
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        uint32_t b = tf;
#pragma unroll
        for (int x = 0; x < kEW; ++x) {
            const uint32_t c = lds[q * kEW + x];
            b += x < wv ? c : 0u;
            tf += c;
        }
        before[q] = b + lanes_below(fm[q]);
    }
    __syncthreads();  // lds is free for the next chunk
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
        const int32_t idx = q * kEThreads + (int32_t)threadIdx.x;  // entries before, in the chunk
        if (e0 + idx >= e1) break;
        if (cnt[q] == 0) {
            const uint32_t f = of + before[q];
            uint4 *d = reinterpret_cast<uint4 *>(s.fdst + (size_t)f * MP);
#pragma unroll
            for (int v = 0; v < MV; ++v) d[v] = rec[q][v];
            rank_s[vec_dword<M % 4>(rec[q][M / 4])] = k;
        } else {
            const uint32_t u = ou + (uint32_t)idx - before[q];
            uint4 *d = reinterpret_cast<uint4 *>(s.udst + (size_t)u * MP);
#pragma unroll
            for (int v = 0; v < MV; ++v) d[v] = rec[q][v];
            s.rdst[u] = run[q];
            s.cdst[u] = cnt[q];
        }
    }
    *nf = tf;
    *nu = (uint32_t)max(e1 - e0, 0) - tf;
}

// Split, writing pass of one item, at the offsets the counting pass scanned.
template <int M>
__device__ void item_splitw(const EInst &I, int32_t k, int32_t n, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const LevelLists s = level_lists(w, L, k);
    const uint32_t *spc = at<uint32_t>(w, L.spc);
    const int32_t e0 = t * kESplit, e1 = min(e0 + kESplit, min(n, I.N));
    uint32_t nf, nu;
    split_chunk<M>(s, k, e0, e1, ld(&spc[2 * t]), ld(&spc[2 * t + 1]), at<int32_t>(w, L.rank_s),
                   smem, &nf, &nu);
}

// Whether level k's front x remaining decrements run over front tables (the
// choice the split's epilogue makes: not when the peeling ends or the one-item
// tail takes over).
__device__ __forceinline__ bool level_uses_tables(const EInst &I, int32_t F, int32_t U) {
    return I.bit_peel && F > 0 && U > 0 && !(U <= I.tail_max && F <= I.tail_front);
}

// Whole split of a short list in one item; writes the level sizes, and the
// front's block tables when the decrements will use them (one stage less).
template <int M>
__device__ void item_split1(const EInst &I, int32_t k, int32_t n, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const LevelLists s = level_lists(w, L, k);
    n = min(n, I.N);
    uint32_t of = 0, ou = 0;
    for (int32_t e0 = 0; e0 < n; e0 += kESplit) {
        uint32_t nf, nu;
        split_chunk<M>(s, k, e0, min(e0 + kESplit, n), of, ou, at<int32_t>(w, L.rank_s), smem, &nf,
                       &nu);
        of += nf;
        ou += nu;
    }
    if (threadIdx.x == 0) {
        at<int32_t>(w, L.fsize)[k] = (int32_t)of;
        at<int32_t>(w, L.usize)[k] = (int32_t)ou;
    }
    if (level_uses_tables(I, (int32_t)of, (int32_t)ou)) {
        __syncthreads();  // every wave's front records are written; the scan scratch is free
        const uint32_t *fk = at<uint32_t>(w, (k & 1) ? L.fk1 : L.fk0);
        const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
        const int32_t nblk = (int32_t)cdiv(of, kBlk);
        for (int32_t b = wv; b < nblk; b += kEThreads / kWave)
            build_block<M, true>(fk, (int32_t)of, at<uint32_t>(w, L.tabs), b,
                                 reinterpret_cast<int32_t *>(smem) + wv * kBlk);
    }
}

// a2 tail: every remaining level of a short list in one item, with block
// barriers only.  Starts after the split of level k (F_k and U_k in the
// level-k lists); per level: F_k x U_k decrements (front chunks staged in
// LDS; each remaining point belongs to one lane of a pass, so plain updates
// suffice), then the split of level k + 1.  Writes the level sizes and the
// number of fronts.
template <int M>
__device__ void item_peel_tail(const EInst &I, int32_t k, uint32_t *smem) {
    const ELayout &L = I.L;
    constexpr int MP = rec_stride(M);
    constexpr int IC = 4096 / MP;  // front records per LDS chunk (16 KiB)
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    int32_t *fsize = at<int32_t>(w, L.fsize), *usize = at<int32_t>(w, L.usize);
    int32_t *rank_s = at<int32_t>(w, L.rank_s);
    uint32_t *lrec = smem;         // [IC * MP]
    uint32_t *lds = smem + 4096;   // scan scratch
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    int32_t nf = ld(&fsize[k]), nu = ld(&usize[k]);
    for (;;) {
        const bool odd = (k & 1) != 0;
        const uint32_t *fk = at<uint32_t>(w, odd ? L.fk1 : L.fk0);
        const uint32_t *uk = at<uint32_t>(w, odd ? L.uk1 : L.uk0);
        const int32_t *urun = at<int32_t>(w, odd ? L.urun1 : L.urun0);
        int32_t *ucnt = at<int32_t>(w, odd ? L.ucnt1 : L.ucnt0);
        // each front chunk is staged once and swept over every remaining tile
        // whose runs it can reach; the counts of a tile's points belong to one
        // lane each, so the chunk's decrements are plain updates
        for (int32_t f0 = 0; f0 < nf; f0 += IC) {
            const int32_t f1 = min(f0 + IC, nf);
            const int32_t fpos = (int32_t)ld(&fk[(size_t)f0 * MP + M]);
            __syncthreads();  // the previous chunk is consumed
            stage_recs<MP>(lrec, fk + (size_t)f0 * MP, f1 - f0);
            __syncthreads();
            for (int32_t j0 = 0; j0 < nu; j0 += kJT) {
                const int32_t jbase = j0 + wv * kWave * kT;
                if (jbase >= nu) break;
                const int32_t run_hi = ld(&urun[min(jbase + kWave * kT - 1, nu - 1)]);
                if (fpos >= run_hi) continue;  // the chunk starts after these runs
                const int32_t run_lo = ld(&urun[jbase]);
                uint32_t kj[kT][M];
                int32_t run[kT], cin[kT];
#pragma unroll
                for (int t = 0; t < kT; ++t) {
                    const int32_t q = jbase + t * kWave + lane;
                    cin[t] = 0;
                    if (q < nu) {
#pragma unroll
                        for (int kk = 0; kk < M; ++kk) kj[t][kk] = uk[(size_t)q * MP + kk];
                        run[t] = urun[q];
                    } else {
#pragma unroll
                        for (int kk = 0; kk < M; ++kk) kj[t][kk] = 0u;
                        run[t] = 0;
                    }
                }
                tile_rows_bounded<M>(lrec, f1 - f0, run_lo, run_hi, kj, run, cin);
#pragma unroll
                for (int t = 0; t < kT; ++t) {
                    const int32_t q = jbase + t * kWave + lane;
                    if (q < nu && cin[t]) ucnt[q] -= cin[t];
                }
            }
        }
        __syncthreads();
        const LevelLists s = level_lists(w, L, k + 1);
        uint32_t of = 0, ou = 0;
        for (int32_t e0 = 0; e0 < nu; e0 += kESplit) {
            uint32_t a, b;
            split_chunk<M>(s, k + 1, e0, min(e0 + kESplit, nu), of, ou, rank_s, lds, &a, &b);
            of += a;
            ou += b;
        }
        ++k;
        if (threadIdx.x == 0) {
            fsize[k] = (int32_t)of;
            usize[k] = (int32_t)ou;
        }
        nf = (int32_t)of;
        nu = (int32_t)ou;
        if (nu == 0 || nf == 0) break;  // nf == 0 with nu > 0 cannot happen; flagged below
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        sc->num_fronts = k + 1;
        if (nu != 0) atomicOr(&sc->err, (uint32_t)kErrInternal);
    }
}

// a2 for two objectives: the points are in lexicographic (key_1, key_2)
// order, so every earlier point has key_1 <= the current one, and an earlier
// point dominates the current point p iff its key_2 is <= p's and it is not
// identical to p (identical points are adjacent and share a rank).  The rank is
// one more than the largest rank among p's dominators.  T2[r], the smallest
// key_2 among points of rank r so far, never decreases with r, so the
// dominators before a batch of 64 points contribute #{r : T2[r] <= key_2(p)}
// (a binary search per lane); dominators inside the batch are folded in order,
// one broadcast per point.  The batch then lowers T2 of its ranks.  One wave,
// one ordered pass; ranks equal the peeling levels.
template <int M>
__device__ void item_rank2(const EInst &I, uint32_t *smem) {
    if constexpr (M != 2) return;  // only two-objective instances take this stage
    const ELayout &L = I.L;
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t N = I.N;
    const uint32_t *recs = at<uint32_t>(w, L.recs);  // [key_1, key_2, position, 0]
    int32_t *rank_s = at<int32_t>(w, L.rank_s);
    constexpr int CAP = kESmem / 2;
    uint32_t *T2 = smem;         // [CAP]
    uint32_t *cnt = smem + CAP;  // [CAP] front sizes
    if (threadIdx.x >= kWave) return;
    const int lane = (int)lane_id();
    int32_t nf = 0;
    bool overflow = false;
    uint32_t pa = 0, pb = 0;  // last point of the previous batch and its rank
    int32_t prank = -1;
    for (int32_t base = 0; base < N; base += kWave) {
        const int32_t p = base + lane;
        const bool valid = p < N;
        const uint32_t a = valid ? recs[(size_t)p * 4] : 0xffffffffu;
        const uint32_t b = valid ? recs[(size_t)p * 4 + 1] : 0xffffffffu;
        // earlier batches: number of fronts with T2 <= b (T2 is non-decreasing)
        int32_t lo = 0, hi = nf;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (T2[mid] <= b) lo = mid + 1; else hi = mid;
        }
        int32_t r = lo;
        // a run of points identical to the previous batch's last one keeps its rank
        if (prank >= 0 && a == pa && b == pb) r = prank;
        // earlier points of this batch, in order (point s is final when folded)
        const int32_t n_here = min(kWave, N - base);
        for (int32_t s = 0; s < n_here; ++s) {
            const int32_t rs = __builtin_amdgcn_readlane(r, s);
            const uint32_t as = __builtin_amdgcn_readlane(a, s);
            const uint32_t bs = __builtin_amdgcn_readlane(b, s);
            if (lane > s && bs <= b && !(as == a && bs == b)) r = max(r, rs + 1);
        }
        int32_t top = valid ? r + 1 : 0;
        for (int o = 32; o > 0; o >>= 1) top = max(top, __shfl_xor(top, o, 64));
        if (top > CAP) { overflow = true; break; }
        for (int32_t q = nf + lane; q < top; q += kWave) {
            T2[q] = 0xffffffffu;
            cnt[q] = 0u;
        }
        nf = max(nf, top);
        if (valid) {
            atomicMin(&T2[r], b);
            atomicAdd(&cnt[r], 1u);
            rank_s[p] = r;
        }
        const int32_t last = n_here - 1;
        pa = __builtin_amdgcn_readlane(a, last);
        pb = __builtin_amdgcn_readlane(b, last);
        prank = __builtin_amdgcn_readlane(r, last);
    }
    int32_t *fsize = at<int32_t>(w, L.fsize);
    if (!overflow)
        for (int32_t r = lane; r < nf; r += kWave) fsize[r] = (int32_t)cnt[r];
    if (lane == 0) {
        sc->rank2_overflow = overflow ? 1 : 0;
        sc->num_fronts = overflow ? 0 : nf;
    }
}

// a2: F_k x U_k decrements for one (front chunk, remaining tile) item.
template <int M>
__device__ void item_phase_a(const EInst &I, int32_t k, int32_t IC, int32_t nJT,
                             int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    constexpr int MP = rec_stride(M);
    char *w = I.ws;
    const int32_t *fsize = at<int32_t>(w, L.fsize);
    const int32_t *usize = at<int32_t>(w, L.usize);
    const int32_t nf = ld(&fsize[k]), nu = ld(&usize[k]);
    const bool odd = (k & 1) != 0;
    const uint32_t *fk = at<uint32_t>(w, odd ? L.fk1 : L.fk0);
    const uint32_t *uk = at<uint32_t>(w, odd ? L.uk1 : L.uk0);
    const int32_t *urun = at<int32_t>(w, odd ? L.urun1 : L.urun0);
    int32_t *ucnt = at<int32_t>(w, odd ? L.ucnt1 : L.ucnt0);
    const int32_t ic = t / nJT, jt = t % nJT;
    const int32_t f0 = ic * IC, f1 = min(f0 + IC, nf);
    const int32_t tile_last = min(jt * kJT + kJT - 1, nu - 1);
    if ((int32_t)ld(&fk[(size_t)f0 * MP + M]) >= ld(&urun[tile_last])) return;
    stage_recs<MP>(smem, fk + (size_t)f0 * MP, f1 - f0);
    __syncthreads();
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    const int32_t jbase = jt * kJT + wv * kWave * kT;
    if (jbase >= nu) return;
    uint32_t kj[kT][M];
    int32_t run[kT], cin[kT];
#pragma unroll
    for (int tt = 0; tt < kT; ++tt) {
        const int32_t q = jbase + tt * kWave + lane;
        cin[tt] = 0;
        if (q < nu) {
#pragma unroll
            for (int kk = 0; kk < M; ++kk) kj[tt][kk] = uk[(size_t)q * MP + kk];
            run[tt] = urun[q];
        } else {
#pragma unroll
            for (int kk = 0; kk < M; ++kk) kj[tt][kk] = 0u;
            run[tt] = 0;
        }
    }
    const int32_t qlast = min(jbase + kWave * kT - 1, nu - 1);
    const int32_t run_lo = ld(&urun[jbase]);
    const int32_t run_hi = ld(&urun[qlast]);
    tile_rows_bounded<M>(smem, f1 - f0, run_lo, run_hi, kj, run, cin);
#pragma unroll
    for (int tt = 0; tt < kT; ++tt) {
        const int32_t q = jbase + tt * kWave + lane;
        if (q < nu && cin[tt]) atomicSub(&ucnt[q], cin[tt]);
    }
}

// a2, block-bitset form: tables of the front F_k, one block of 64 entries per
// wave (the tables of the dominance counts are free again by now).
template <int M>
__device__ void item_build_f(const EInst &I, int32_t k, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const int32_t nf = ld(&at<int32_t>(w, L.fsize)[k]);
    const uint32_t *fk = at<uint32_t>(w, (k & 1) ? L.fk1 : L.fk0);
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    build_block<M, true>(fk, nf, at<uint32_t>(w, L.tabs), t * (kEThreads / kWave) + wv,
                         reinterpret_cast<int32_t *>(smem) + wv * kBlk);
}

// a2, block-bitset form: one (chunk of cb front tables, group of remaining
// tiles) item of level k; p0 = cb, p1 = tile groups.  Remaining-list tiles per
// item (whole table chunks per item): 1, 2, 4 and 8 tiles took 18.1, 14.4,
// 14.1 and 15.2 ms per launch on the mixed batch when first measured, and
// splitting small levels into smaller chunks was slower still; with the
// coalesced level split, 2, 4, 8 and 16 tiles took 10.7-10.8, 10.35-10.41,
// 10.24-10.36 and 10.34-10.56 ms.
constexpr int kLevelTiles = 8;
static_assert(kEThreads == kFwdThreads, "engine work-groups run the bitset bodies");

template <int M>
__device__ void item_phase_a_bits(const EInst &I, int32_t k, int32_t cb, int32_t ngroups, int32_t t,
                                  uint32_t *smem) {
    static_assert(level_chunk<M>() * blk_stride(M) <= kESmem,
                  "a chunk of tables fits the worker's LDS");
    const ELayout &L = I.L;
    char *w = I.ws;
    const int32_t nf = ld(&at<int32_t>(w, L.fsize)[k]);
    const int32_t nu = ld(&at<int32_t>(w, L.usize)[k]);
    const bool odd = (k & 1) != 0;
    const int32_t nblk = (int32_t)cdiv(nf, kBlk);
    const int32_t ic = t / ngroups, jg = t % ngroups;
    const int32_t b0 = ic * cb;
    fwd_level_item<M, kLevelTiles>(at<const uint32_t>(w, L.tabs), b0, min(cb, nblk - b0),
                                   at<const uint32_t>(w, odd ? L.uk1 : L.uk0),
                                   at<const int32_t>(w, odd ? L.urun1 : L.urun0), nu,
                                   at<int32_t>(w, odd ? L.ucnt1 : L.ucnt0), jg * kLevelTiles, smem);
}

// Ranks and counts back to the original order.
__device__ void item_orig(const EInst &I, int32_t t) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const uint32_t *sval = at<uint32_t>(w, (sort_passes(I) & 1) ? L.sval1 : L.sval0);
    const int32_t *rank_s = at<int32_t>(w, L.rank_s);
    const int32_t *din = at<int32_t>(w, L.din), *dout = at<int32_t>(w, L.dout);
    int32_t *rank = I.rank ? I.rank : at<int32_t>(w, L.rank);
    for (int q = 0; q < kEChunk / kEThreads; ++q) {
        const int32_t p = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        if (p >= I.N) break;
        const uint32_t i = sval[p];
        rank[i] = rank_s[p];
        if (I.dom_in) I.dom_in[i] = din[p];
        if (I.dom_out) I.dom_out[i] = dout[p];
    }
}

// a4: extreme-point (ASF argmin per axis) and nadir partials of one chunk.
template <int M>
__device__ void item_ext(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t *rank = I.rank ? I.rank : at<int32_t>(w, L.rank);
    const int32_t l = ld(&sc->last_front);
    double z[M], best[M], nad[M];
    int32_t bidx[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        z[k] = (double)key_to_float(ld(&sc->min_key[k]));
        best[k] = DBL_MAX;
        bidx[k] = 0x7fffffff;
        nad[k] = 0.0;
    }
    for (int q = 0; q < kEChunk / kEThreads; ++q) {
        const int32_t i = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        if (i >= I.N) break;
        if (rank[i] > l) continue;
        double g[M];
#pragma unroll
        for (int k = 0; k < M; ++k) g[k] = (double)I.objs[(int64_t)i * M + k] - z[k];
        asf_fold<M>(g, M, i, best, bidx, nad);
    }
    double *s_asf = reinterpret_cast<double *>(smem);            // [kWaves][M]
    double *s_nad = s_asf + kWaves * 16;                          // [kWaves][M]
    int32_t *s_idx = reinterpret_cast<int32_t *>(s_nad + kWaves * 16);
    const int wv = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double b = best[j];
        int32_t bi = bidx[j];
        double nd = nad[j];
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(b, o, 64);
            const int32_t oi = __shfl_xor(bi, o, 64);
            if (ob < b || (ob == b && oi < bi)) { b = ob; bi = oi; }
            const double on = __shfl_xor(nd, o, 64);
            nd = on > nd ? on : nd;
        }
        if (lane_id() == 0) { s_asf[wv * 16 + j] = b; s_idx[wv * 16 + j] = bi; s_nad[wv * 16 + j] = nd; }
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        const int j = threadIdx.x;
        double b = s_asf[j];
        int32_t bi = s_idx[j];
        double nd = s_nad[j];
        for (int q = 1; q < kWaves; ++q) {
            const double a = s_asf[q * 16 + j];
            const int32_t ai = s_idx[q * 16 + j];
            if (a < b || (a == b && ai < bi)) { b = a; bi = ai; }
            nd = s_nad[q * 16 + j] > nd ? s_nad[q * 16 + j] : nd;
        }
        at<double>(w, L.p_asf)[(size_t)t * M + j] = b;
        at<int32_t>(w, L.p_idx)[(size_t)t * M + j] = bi;
        at<double>(w, L.p_nad)[(size_t)t * M + j] = nd;
    }
}

// a6/a7: association of one point per thread; the float32 unit references
// pass through LDS in chunks, twice (maximum, then candidates).
static_assert(8192 + 2 * kLdsNicheRefs <= kESmem, "association LDS: reference chunk + tallies");

template <int M>
__device__ void item_assoc(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    constexpr int HC = 8192 / M;  // references per LDS chunk
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t H = I.H;
    const float *r32 = at<float>(w, L.rhat32);
    const double *r64 = at<double>(w, L.rhat64);
    float *lr = reinterpret_cast<float *>(smem);
    const int32_t l = ld(&sc->last_front);
    const int32_t i = t * kEThreads + (int32_t)threadIdx.x;
    const bool inr = i < I.N;
    const int32_t *rank = I.rank ? I.rank : at<int32_t>(w, L.rank);
    const int32_t r = inr ? rank[i] : 0x7fffffff;
    const bool active = inr && r <= l;
    double z[M], a[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        z[k] = ldd(&sc->z[k]);
        a[k] = ldd(&sc->a[k]);
    }
    double fp[M];
    float y[M];
    float l1 = 0.0f;
    if (active) l1 = normalise_point<M>(I.objs + (int64_t)i * M, z, a, fp, y);
    else {
#pragma unroll
        for (int k = 0; k < M; ++k) { fp[k] = 0.0; y[k] = 0.0f; }
    }
    double d1 = DBL_MAX, d2 = DBL_MAX;
    int32_t best = 0;
    const int32_t hm = H * M, hm2 = (hm + 1) & ~1;
    if (hm2 + 2 * hm <= 8192) {
        // both unit-reference forms in LDS (the float64 re-scoring then reads
        // no global memory); the same screening as the single path
        double *lr64 = reinterpret_cast<double *>(smem + hm2);
        for (int32_t q = threadIdx.x; q < hm; q += kEThreads) {
            lr[q] = r32[q];
            lr64[q] = r64[q];
        }
        __syncthreads();
        if (active) associate_point<M>(fp, y, l1, lr, lr64, H, best, d1, d2);
    } else {
        float smax = -FLT_MAX;
        for (int32_t c0 = 0; c0 < H; c0 += HC) {
            const int32_t hc = min(HC, H - c0);
            __syncthreads();
            for (int32_t q = threadIdx.x; q < hc * M; q += kEThreads) lr[q] = r32[(size_t)c0 * M + q];
            __syncthreads();
            for (int32_t j = 0; j < hc; ++j) {
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k) s = __fmaf_rn(y[k], lr[j * M + k], s);
                smax = s > smax ? s : smax;
            }
        }
        const float thr = smax - fp32_band<M>(l1);
        for (int32_t c0 = 0; c0 < H; c0 += HC) {
            const int32_t hc = min(HC, H - c0);
            if (c0 > 0 || hc < H) {  // the single-chunk case still holds the chunk
                __syncthreads();
                for (int32_t q = threadIdx.x; q < hc * M; q += kEThreads) lr[q] = r32[(size_t)c0 * M + q];
                __syncthreads();
            }
            if (active) {
                for (int32_t j = 0; j < hc; ++j) {
                    float s = 0.0f;
#pragma unroll
                    for (int k = 0; k < M; ++k) s = __fmaf_rn(y[k], lr[j * M + k], s);
                    if (s < thr) continue;
                    const double d = line_distance<M>(fp, r64 + (size_t)(c0 + j) * M);
                    if (d < d1) { d2 = d1; d1 = d; best = c0 + j; }
                    else if (d < d2) { d2 = d; }
                }
            }
        }
    }
    int32_t *niche = I.niche ? I.niche : at<int32_t>(w, L.niche);
    double *dist64 = at<double>(w, L.dist64);
    uint8_t *selflag = at<uint8_t>(w, L.selflag);
    int cls = -1;
    if (active) {
        niche[i] = best;
        if (I.dist) I.dist[i] = (float)d1;
        dist64[i] = d1;
        if (near_tie(d1, d2)) atomicAdd(&sc->near_ties, 1);
        cls = r < l ? 0 : 1;
        selflag[i] = r < l ? 1 : 0;
    } else if (inr) {
        niche[i] = -1;
        if (I.dist) I.dist[i] = -1.0f;
        dist64[i] = -1.0;
        selflag[i] = 0;
    }
    // the tallies sit past the reference chunk, which other waves may still read
    niche_count_block(H, cls, best, at<int32_t>(w, L.rho), at<int32_t>(w, L.bcount),
                      reinterpret_cast<int32_t *>(smem) + 8192);
}

// Last-front members into their reference buckets.
__device__ void item_bscat(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t l = ld(&sc->last_front);
    const int32_t *rank = I.rank ? I.rank : at<int32_t>(w, L.rank);
    const int32_t *niche = I.niche ? I.niche : at<int32_t>(w, L.niche);
    const double *dist64 = at<double>(w, L.dist64);
    int32_t *bcursor = at<int32_t>(w, L.bcursor);
    double *bd = at<double>(w, L.bd);
    int32_t *bi = at<int32_t>(w, L.bi);
    for (int q = 0; q < kEChunk / kEThreads; ++q) {
        const int32_t i = t * kEChunk + q * kEThreads + (int32_t)threadIdx.x;
        const bool member = i < I.N && rank[i] == l;
        const int32_t b = member ? niche[i] : 0;
        const int32_t slot =
            bucket_slot_block(I.H, member, b, bcursor, reinterpret_cast<int32_t *>(smem));
        if (member) {
            bd[slot] = dist64[i];
            bi[slot] = i;
        }
    }
}

// a8: t_i = members of the same reference with smaller (distance, index);
// pick when (rho + t, reference) is below the threshold.
__device__ void item_brank(const EInst &I, int32_t t) {
    const ELayout &L = I.L;
    char *w = I.ws;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t s = t * kEThreads + (int32_t)threadIdx.x;
    if (s >= ld(&sc->last_front_size)) return;
    const int32_t *niche = I.niche ? I.niche : at<int32_t>(w, L.niche);
    const int32_t *rho = at<int32_t>(w, L.rho);
    const int32_t *bstart = at<int32_t>(w, L.bstart);
    const double *bd = at<double>(w, L.bd);
    const int32_t *bi = at<int32_t>(w, L.bi);
    const double d = bd[s];
    const int32_t i = bi[s];
    const int32_t j = niche[i];
    const int32_t b0 = bstart[j], b1 = bstart[j + 1];
    int32_t tt = 0;
    for (int32_t m = b0; m < b1; ++m) {
        const double dm = bd[m];
        const int32_t im = bi[m];
        tt += (dm < d || (dm == d && im < i)) ? 1 : 0;
    }
    const int64_t lev = (int64_t)rho[j] + tt;
    const int64_t V = ld(&sc->level_V);
    if (lev < V || (lev == V && j < ld(&sc->ref_thr))) at<uint8_t>(w, L.selflag)[i] = 1;
}

__device__ void item_cmpc(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const uint8_t *flag = at<uint8_t>(w, L.selflag);
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < kECmp / kEThreads; ++it) {
        const int32_t p = t * kECmp + it * kEThreads + (int32_t)threadIdx.x;
        if (p < I.N && flag[p]) ++c;
    }
    c = wave_sum(c);
    if (lane_id() == 0) smem[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int q = 0; q < kWaves; ++q) s += smem[q];
        at<uint32_t>(w, L.cmpc)[t] = s;
    }
}

__device__ void item_cmpw(const EInst &I, int32_t t, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const uint8_t *flag = at<uint8_t>(w, L.selflag);
    uint32_t off = ld(&at<uint32_t>(w, L.cmpc)[t]);
    for (int it = 0; it < kECmp / kEThreads; ++it) {
        const int32_t p = t * kECmp + it * kEThreads + (int32_t)threadIdx.x;
        const uint32_t f = (p < I.N && flag[p]) ? 1u : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(f, smem, &tot);
        if (f && (int64_t)(off + ex) < I.K) I.selected[off + ex] = p;
        off += tot;
    }
}

template <int M>
__device__ void run_item(const EInst &I, int32_t stage, int32_t arg, int32_t n,
                         int32_t p0, int32_t p1, int32_t t, uint32_t *smem) {
    switch (stage) {
        case kSPrep: item_prep<M>(I, t, smem); break;
        case kSHist: item_hist(I, arg, t, smem); break;
        case kSScat: item_scat(I, arg, t, smem); break;
        case kSRecs: item_recs<M>(I, t); break;
        case kSDom: item_dom<M>(I, t, smem); break;
        case kSSplitC: item_splitc(I, arg, n, t, smem); break;
        case kSSplitW: item_splitw<M>(I, arg, n, t, smem); break;
        case kSSplit1: item_split1<M>(I, arg, n, smem); break;
        case kSPeelTail: item_peel_tail<M>(I, arg, smem); break;
        case kSRank2: item_rank2<M>(I, smem); break;
        case kSPhaseA:
            if (I.bit_peel) item_phase_a_bits<M>(I, arg, p0, p1, t, smem);
            else item_phase_a<M>(I, arg, p0, p1, t, smem);
            break;
        case kSBuildF: item_build_f<M>(I, arg, t, smem); break;
        case kSOrig: item_orig(I, t); break;
        case kSExt: item_ext<M>(I, t, smem); break;
        case kSAssoc: item_assoc<M>(I, t, smem); break;
        case kSBScat: item_bscat(I, t, smem); break;
        case kSBRank: item_brank(I, t); break;
        case kSCmpC: item_cmpc(I, t, smem); break;
        case kSCmpW: item_cmpw(I, t, smem); break;
        default: break;
    }
}

// ---------------------------------------------------------------------------
// Stage epilogues (whole block; the instance is owned by this block until
// the next stage is published)
// ---------------------------------------------------------------------------

// Exclusive scan in place of n uint32 values at stride `stride` (block-wide);
// returns the total.
__device__ uint32_t scan_strided(uint32_t *v, int32_t n, int stride, uint32_t *lds) {
    uint32_t run = 0;
    for (int32_t base = 0; base < n; base += kEThreads) {
        const int32_t e = base + (int32_t)threadIdx.x;
        const uint32_t x = e < n ? ld(&v[(size_t)e * stride]) : 0u;
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(x, lds, &tot);
        if (e < n) v[(size_t)e * stride] = run + ex;
        run += tot;
    }
    return run;
}

// a5 epilogue: reduce the extreme-point partials, solve for the intercepts.
template <int M>
__device__ void epi_solve(const EInst &I, EScal *sc, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const int32_t nparts = (int32_t)cdiv(I.N, kEChunk);
    int32_t *s_e = reinterpret_cast<int32_t *>(smem);
    double *s_nad = reinterpret_cast<double *>(smem + 32);
    if (threadIdx.x < kWave) {
        const double *p_asf = at<double>(w, L.p_asf), *p_nad = at<double>(w, L.p_nad);
        const int32_t *p_idx = at<int32_t>(w, L.p_idx);
        for (int j = 0; j < M; ++j) {
            double b = DBL_MAX;
            int32_t bi = 0x7fffffff;
            double nd = 0.0;
            for (int32_t q = threadIdx.x; q < nparts; q += kWave) {
                const double a = p_asf[(size_t)q * M + j];
                const int32_t ai = p_idx[(size_t)q * M + j];
                if (a < b || (a == b && ai < bi)) { b = a; bi = ai; }
                const double nn = p_nad[(size_t)q * M + j];
                nd = nn > nd ? nn : nd;
            }
            for (int o = 32; o > 0; o >>= 1) {
                const double ob = __shfl_xor(b, o, 64);
                const int32_t oi = __shfl_xor(bi, o, 64);
                if (ob < b || (ob == b && oi < bi)) { b = ob; bi = oi; }
                const double on = __shfl_xor(nd, o, 64);
                nd = on > nd ? on : nd;
            }
            if (threadIdx.x == 0) { s_e[j] = bi; s_nad[j] = nd; }
        }
    }
    __syncthreads();
    if (threadIdx.x < kWave) {
        double z[M], a[M];
#pragma unroll
        for (int k = 0; k < M; ++k) z[k] = (double)key_to_float(ld(&sc->min_key[k]));
        const int fb = solve_intercepts_wave<M>(I.objs, s_e, s_nad, z, a);
        if (threadIdx.x == 0) {
            for (int k = 0; k < M; ++k) {
                sc->z[k] = z[k];
                sc->a[k] = a[k];
            }
            sc->fallback = fb;
        }
    }
    __syncthreads();
}

// a8 plan epilogue: bucket offsets of the last front by reference, and the
// selection threshold V* = max{V : C(V) <= R}, C(V) = sum_j clamp(V - rho_j,
// 0, b_j); the remaining R - C(V*) picks are the level-V* members of the
// lowest-indexed references.
__device__ void epi_niche_plan(const EInst &I, EScal *sc, uint32_t *smem) {
    const ELayout &L = I.L;
    char *w = I.ws;
    const int32_t H = I.H;
    const int32_t *rho = at<int32_t>(w, L.rho);
    const int32_t *bcount = at<int32_t>(w, L.bcount);
    int32_t *bstart = at<int32_t>(w, L.bstart);
    int32_t *bcursor = at<int32_t>(w, L.bcursor);
    uint32_t *lds = smem;
    int64_t *red = reinterpret_cast<int64_t *>(smem + 32);
    int32_t *s_thr = reinterpret_cast<int32_t *>(smem + 64);
    const int64_t R = ld(&sc->R);
    uint32_t run = 0;
    int64_t vmax = 0;
    for (int32_t base = 0; base < H; base += kEThreads) {
        const int32_t j = base + (int32_t)threadIdx.x;
        const uint32_t v = j < H ? (uint32_t)ld(&bcount[j]) : 0u;
        if (j < H) {
            const int64_t top = (int64_t)ld(&rho[j]) + (int64_t)v;
            vmax = top > vmax ? top : vmax;
        }
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(v, lds, &tot);
        if (j < H) { bstart[j] = (int32_t)(run + ex); bcursor[j] = (int32_t)(run + ex); }
        run += tot;
    }
    if (threadIdx.x == 0) bstart[H] = (int32_t)run;
    vmax = wave_max(vmax);
    if (lane_id() == 0) red[threadIdx.x / kWave] = vmax;
    __syncthreads();
    int64_t hi = 0;
    for (int q = 0; q < kWaves; ++q) hi = red[q] > hi ? red[q] : hi;
    __syncthreads();
    auto count_below = [&](int64_t V) {
        int64_t c = 0;
        for (int32_t j = threadIdx.x; j < H; j += kEThreads) {
            int64_t tt = V - ld(&rho[j]);
            tt = tt < 0 ? 0 : tt;
            const int64_t bc = ld(&bcount[j]);
            c += tt < bc ? tt : bc;
        }
        c = wave_sum(c);
        if (lane_id() == 0) red[threadIdx.x / kWave] = c;
        __syncthreads();
        int64_t tot = 0;
        for (int q = 0; q < kWaves; ++q) tot += red[q];
        __syncthreads();
        return tot;
    };
    int64_t lo = 0;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) >> 1;
        if (count_below(mid) <= R) lo = mid; else hi = mid - 1;
    }
    const int64_t V = lo;
    const int64_t rem = R - count_below(V);
    if (threadIdx.x == 0) *s_thr = rem <= 0 ? 0 : H;
    __syncthreads();
    if (rem > 0) {
        uint32_t seen = 0;
        for (int32_t base = 0; base < H; base += kEThreads) {
            const int32_t j = base + (int32_t)threadIdx.x;
            uint32_t has = 0;
            if (j < H) {
                const int64_t rj = ld(&rho[j]);
                has = (rj <= V && V < rj + (int64_t)ld(&bcount[j])) ? 1u : 0u;
            }
            uint32_t tot;
            const uint32_t ex = block_exclusive_scan(has, lds, &tot);
            if (has && (int64_t)(seen + ex) == rem - 1) *s_thr = j + 1;
            seen += tot;
            if ((int64_t)seen >= rem) break;  // uniform: seen is block-wide
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        sc->level_V = (int32_t)V;
        sc->ref_thr = *s_thr;
    }
}

__device__ void finalize_info(const EInst &I, EScal *sc) {
    uint32_t e = ld(&sc->err);
    if (e == 0 && (int64_t)ld(&sc->n_selected) != I.K) e |= kErrInternal;
    if (!I.info) return;
    nsga3_info v;
    v.status = e == 0 ? NSGA3_OK
               : (e & (kErrNonfiniteObj | kErrBadRef)) ? NSGA3_E_NONFINITE
                                                       : NSGA3_E_HIP;
    v.last_front = ld(&sc->last_front);
    v.num_fronts = ld(&sc->num_fronts);
    v.last_front_size = ld(&sc->last_front_size);
    v.num_from_last = (int32_t)ld(&sc->R);
    v.intercept_fallback = ld(&sc->fallback);
    v.near_ties = ld(&sc->near_ties);
    v.reserved = (int32_t)e;
    *I.info = v;
}

// Runs the epilogue of the stage that just completed and publishes the next
// stage with at least one item (or marks the instance done).
template <int M>
__device__ void advance(const EInst &I, EState *S, EGlobal *g, int32_t stop_stage, uint32_t *smem) {
    constexpr int MP = rec_stride(M);
    char *w = I.ws;
    const ELayout &L = I.L;
    EScal *sc = at<EScal>(w, L.scal);
    const int32_t N = I.N;
    int32_t stage = ld(&S->stage), arg = ld(&S->arg), n = ld(&S->n);
    int32_t p0 = 0, p1 = 0;
    int64_t items = 0;
    // level `level` of the peeling starts with a split of a list of `len` entries
    auto begin_level = [&](int32_t level, int32_t len) {
        arg = level;
        n = len;
        if (n <= kESplitOne) { stage = kSSplit1; items = 1; }
        else { stage = kSSplitC; items = cdiv(n, kESplit); }
    };
    // bitset decrements of level arg over the front's tables
    auto to_phase_a = [&](int32_t F, int32_t U) {
        constexpr int CB = level_chunk<M>();
        stage = kSPhaseA;
        n = U;
        p0 = CB;                                              // tables per item
        p1 = (int32_t)cdiv(cdiv(U, kTileJ), kLevelTiles);  // tile groups
        items = cdiv(cdiv(F, kBlk), CB) * p1;
    };
    // after the split of level arg: F fronts, U remaining (block-uniform);
    // tables_ready: the split item built the front's tables already
    auto after_split = [&](int32_t F, int32_t U, bool tables_ready) {
        if (threadIdx.x == 0) {
            // a3: the first level whose cumulative size reaches K
            if (ld(&sc->last_front) < 0 && F > 0) {
                const int64_t cum = ld(&sc->n_before);
                if (cum + (int64_t)F >= I.K) {
                    sc->last_front = arg;
                    sc->last_front_size = F;
                    sc->R = I.K - cum;
                } else {
                    sc->n_before = cum + F;
                }
            }
            if (F <= 0) atomicOr(&sc->err, (uint32_t)kErrInternal);  // impossible for a partial order
            if (U == 0) sc->num_fronts = arg + 1;
        }
        __syncthreads();
        if (F <= 0) {
            stage = kSDone;
        } else if (U == 0) {
            stage = kSOrig;
            items = cdiv(N, kEChunk);
        } else if (U <= I.tail_max && F <= I.tail_front) {
            stage = kSPeelTail;
            items = 1;
        } else if (I.bit_peel) {
            if (tables_ready) {
                to_phase_a(F, U);
            } else {
                stage = kSBuildF;  // then kSPhaseA over the tables
                n = U;
                items = cdiv(cdiv(F, kBlk), kEThreads / kWave);
            }
        } else {
            const int32_t nJT = (int32_t)cdiv(U, kJT);
            int32_t IC = 4096 / MP;
            while (IC > 64 && cdiv(F, IC) * nJT < I.pa_items) IC >>= 1;
            stage = kSPhaseA;
            p0 = IC;
            p1 = nJT;
            n = U;
            items = cdiv(F, IC) * nJT;
        }
    };
    for (;;) {
        if (ld(&sc->err) != 0) {  // outputs are undefined after a device-side error
            stage = kSDone;
            break;
        }
        switch (stage) {
            case kSPrep:
                if (threadIdx.x == 0) {
                    int passes = radix_passes(M);
                    if (M != 2) {  // 8-bit digits of (key - min key): the range's bits
                        const unsigned long long lo = ld(&sc->skey_min), hi = ld(&sc->skey_max);
                        const int bits = hi > lo ? 64 - __clzll((long long)(hi - lo)) : 0;
                        passes = bits <= 8 ? 1 : (bits + 7) / 8;
                    }
                    sc->rs_passes = passes;
                }
                __syncthreads();
                stage = kSHist; arg = 0; items = cdiv(N, kERsTile);
                break;
            case kSHist:
                stage = kSScat; items = cdiv(N, kERsTile);
                break;
            case kSScat:
                if (arg + 1 < ld(&sc->rs_passes)) { stage = kSHist; ++arg; items = cdiv(N, kERsTile); }
                else { stage = kSRecs; items = cdiv(N, kEChunk); }
                break;
            case kSRecs: {
                stage = kSDom;
                const int64_t T = cdiv(N, kJT);
                items = T * (T + 1) / 2;
                break;
            }
            case kSDom:
                if (threadIdx.x == 0) {
                    sc->n_before = 0;
                    sc->last_front = -1;
                }
                __syncthreads();
                begin_level(0, N);
                break;
            case kSSplitC: {
                uint32_t *spc = at<uint32_t>(w, L.spc);
                const int32_t m = (int32_t)cdiv(n, kESplit);
                const uint32_t F = scan_strided(spc, m, 2, smem);
                const uint32_t U = scan_strided(spc + 1, m, 2, smem);
                if (threadIdx.x == 0) {
                    at<int32_t>(w, L.fsize)[arg] = (int32_t)F;
                    at<int32_t>(w, L.usize)[arg] = (int32_t)U;
                }
                __syncthreads();
                stage = kSSplitW; items = m;
                break;
            }
            case kSSplitW:
            case kSSplit1:
                after_split(ld(&at<int32_t>(w, L.fsize)[arg]), ld(&at<int32_t>(w, L.usize)[arg]),
                            stage == kSSplit1);
                break;
            case kSBuildF:
                to_phase_a(ld(&at<int32_t>(w, L.fsize)[arg]), n);
                break;
            case kSPhaseA:
                begin_level(arg + 1, n);
                break;
            case kSRank2:
                if (ld(&sc->rank2_overflow)) {  // too many fronts for the ordered pass
                    begin_level(0, N);
                    break;
                }
                arg = -1;  // every level is still to be counted
                // fall through: a3 over the fronts the pass found
            case kSPeelTail: {
                // a3 for the levels the tail peeled (level arg was counted already)
                if (threadIdx.x == 0) {
                    const int32_t nfr = ld(&sc->num_fronts);
                    const int32_t *fsz = at<int32_t>(w, L.fsize);
                    int64_t cum = ld(&sc->n_before);
                    for (int32_t lv = arg + 1; lv < nfr && ld(&sc->last_front) < 0; ++lv) {
                        const int32_t F = ld(&fsz[lv]);
                        if (cum + (int64_t)F >= I.K) {
                            sc->last_front = lv;
                            sc->last_front_size = F;
                            sc->R = I.K - cum;
                        } else {
                            cum += F;
                        }
                    }
                    sc->n_before = cum;
                }
                __syncthreads();
                stage = kSOrig;
                items = cdiv(N, kEChunk);
                break;
            }
            case kSOrig:
                stage = kSExt; items = cdiv(N, kEChunk);
                break;
            case kSExt:
                epi_solve<M>(I, sc, smem);
                stage = kSAssoc; items = cdiv(N, kEThreads);
                break;
            case kSAssoc:
                epi_niche_plan(I, sc, smem);
                stage = kSBScat; items = cdiv(N, kEChunk);
                break;
            case kSBScat:
                stage = kSBRank; items = cdiv(ld(&sc->last_front_size), kEThreads);
                break;
            case kSBRank:
                stage = kSCmpC; items = cdiv(N, kECmp);
                break;
            case kSCmpC: {
                const uint32_t tot = scan_strided(at<uint32_t>(w, L.cmpc), (int32_t)cdiv(N, kECmp), 1, smem);
                if (threadIdx.x == 0) sc->n_selected = tot;
                __syncthreads();
                stage = kSCmpW; items = cdiv(N, kECmp);
                break;
            }
            case kSCmpW:
            default:
                stage = kSDone;
                break;
        }
        if (stage == kSDone || items > 0) break;
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have reached the L2
    __syncthreads();
    if (threadIdx.x == 0) {
        const bool leave = stage == kSDone || stage == stop_stage;  // done, or parked
        if (stage == kSDone) finalize_info(I, sc);
        S->stage = stage;
        S->arg = arg;
        S->n = n;
        S->p0 = p0;
        S->p1 = p1;
        S->done = 0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // write every wave's stores back
        __hip_atomic_store(&S->word, leave ? 0ull : (uint64_t)items, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
        if (leave)
            __hip_atomic_fetch_add(&g->finished, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Kernels
// ---------------------------------------------------------------------------
__device__ __forceinline__ void stat_add(unsigned long long *p, unsigned long long v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int M>
__global__ __launch_bounds__(kEThreads) void k_engine(const EInst *__restrict__ inst, EState *st,
                                                      int32_t b0, int32_t nb, EGlobal *g,
                                                      EStats *stats, int32_t stop_stage) {
    __shared__ __attribute__((aligned(16))) uint32_t smem[kESmem];
    __shared__ int32_t s_b, s_item;
    __shared__ uint32_t s_total, s_flag;
    const uint32_t lane = lane_id();
    int32_t cursor = (int32_t)(blockIdx.x % (uint32_t)nb);
    bool idle = false;
    long long idle_t0 = 0;
    uint32_t backoff = 1;  // s_sleep units after a search that found nothing
    for (;;) {
        const long long t0 = stats ? wall_clock64() : 0;
        if (threadIdx.x < kWave) {
            int32_t found = -1;
            uint32_t item = 0, total = 0;
            // the instance this block worked on last comes first: its next
            // items are usually ready
            if (lane == 0) {
                const uint64_t wd = lda(&st[b0 + cursor].word);
                if ((uint32_t)(wd >> 32) < (uint32_t)wd) {
                    const uint64_t old = __hip_atomic_fetch_add(&st[b0 + cursor].word, 1ull << 32,
                                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if ((uint32_t)(old >> 32) < (uint32_t)old) {
                        found = cursor;
                        item = (uint32_t)(old >> 32);
                        total = (uint32_t)old;
                    }
                }
            }
            found = __shfl(found, 0, 64);
            // then a scan from the next instance on, 4 x 64 progress words in flight
            const int32_t start = cursor + 1 < nb ? cursor + 1 : 0;
            for (int32_t base = 0; base < nb && found < 0; base += 4 * kWave) {
                uint64_t m[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int32_t off = base + r * kWave + (int32_t)lane;
                    bool ok = false;
                    if (off < nb) {
                        int32_t q = start + off;
                        q -= q >= nb ? nb : 0;
                        const uint64_t wd = lda(&st[b0 + q].word);
                        ok = (uint32_t)(wd >> 32) < (uint32_t)wd;
                    }
                    m[r] = ballot(ok);
                }
                if (lane == 0) {
                    for (int r = 0; r < 4 && found < 0; ++r) {
                        uint64_t mm = m[r];
                        while (mm) {
                            const int l = __builtin_ctzll(mm);
                            mm &= mm - 1;
                            int32_t q = start + base + r * kWave + l;
                            q -= q >= nb ? nb : 0;
                            const uint64_t old = __hip_atomic_fetch_add(
                                &st[b0 + q].word, 1ull << 32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            if ((uint32_t)(old >> 32) < (uint32_t)old) {
                                found = q;
                                item = (uint32_t)(old >> 32);
                                total = (uint32_t)old;
                                break;
                            }
                        }
                    }
                }
                found = __shfl(found, 0, 64);
            }
            if (lane == 0) {
                s_b = found;
                s_item = (int32_t)item;
                s_total = total;
                if (found >= 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            }
        }
        __syncthreads();
        const int32_t b = s_b;
        long long t1 = 0;
        if (stats && threadIdx.x == 0) {
            t1 = wall_clock64();
            stat_add(b < 0 ? &stats->idle : &stats->probe, (unsigned long long)(t1 - t0));
        }
        if (b < 0) {
            if (threadIdx.x == 0) {
                uint32_t stop = 0;
                if (lda(&g->finished) >= (uint32_t)nb || lda(&g->err) != 0) {
                    stop = 1;
                } else {
                    const long long now = wall_clock64();
                    if (!idle) {
                        idle = true;
                        idle_t0 = now;
                    } else if ((unsigned long long)(now - idle_t0) > kIdleLimit) {
                        atomicOr(&g->err, (uint32_t)kErrBarrierTimeout);
                        stop = 1;
                    }
                    for (uint32_t q = 0; q < backoff; ++q) __builtin_amdgcn_s_sleep(8);
                    backoff = backoff < 32u ? 2u * backoff : 32u;
                }
                s_flag = stop;
            }
            __syncthreads();
            if (s_flag) return;
            continue;
        }
        idle = false;
        backoff = 1;
        cursor = b;
        const EInst &I = inst[b0 + b];
        EState *S = st + b0 + b;
        const int32_t stage = ld(&S->stage);
        run_item<M>(I, stage, ld(&S->arg), ld(&S->n), ld(&S->p0), ld(&S->p1), s_item, smem);
        // every wave's stores reach the L2, then one release writes them back
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (threadIdx.x == 0) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t d = __hip_atomic_fetch_add(&S->done, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t last = d + 1 == s_total ? 1u : 0u;
            if (last) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            s_flag = last;
        }
        __syncthreads();
        long long t2 = 0;
        if (stats && threadIdx.x == 0) {
            t2 = wall_clock64();
            stat_add(&stats->item[stage], (unsigned long long)(t2 - t1));
            stat_add(&stats->items[stage], 1ull);
        }
        if (s_flag) {
            advance<M>(I, S, g, stop_stage, smem);
            if (stats && threadIdx.x == 0)
                stat_add(&stats->epilogue[stage], (unsigned long long)(wall_clock64() - t2));
        }
        __syncthreads();
    }
}

// Resets every instance to its first stage and clears the scalars.
__global__ void k_engine_init(const EInst *__restrict__ inst, EState *st, EGlobal *g, int32_t B,
                              int32_t nclass) {
    const int32_t b = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (b < nclass) {
        g[b].finished = 0;
        g[b].err = 0;
    }
    if (b >= B) return;
    const EInst &I = inst[b];
    EScal *sc = at<EScal>(I.ws, I.L.scal);
    sc->err = 0;
    for (int k = 0; k < 16; ++k) {
        sc->min_key[k] = 0xffffffffu;
        sc->z[k] = 0.0;
        sc->a[k] = 1.0;
    }
    sc->skey_min = ~0ull;
    sc->skey_max = 0ull;
    sc->rs_passes = radix_passes(I.M);
    sc->num_fronts = 0;
    sc->last_front = 0;
    sc->last_front_size = 0;
    sc->fallback = 0;
    sc->n_before = 0;
    sc->R = 0;
    sc->near_ties = 0;
    sc->level_V = 0;
    sc->ref_thr = 0;
    sc->n_selected = 0;
    sc->rank2_overflow = 0;
    EState &S = st[b];
    S.stage = kSPrep;
    S.arg = 0;
    S.n = I.N;
    S.p0 = S.p1 = 0;
    S.done = 0;
    S.word = (uint64_t)(cdiv(I.N, kEChunk) + cdiv(I.H, kEThreads));
}

// Dominance counts of parked instances, one (instance, item) per block.  The
// instance tables and records were written by an earlier launch, so plain
// scalar loads are safe here.
template <int M>
__global__ __launch_bounds__(kEThreads) void k_engine_dom(const EInst *__restrict__ inst,
                                                          const EState *__restrict__ st,
                                                          const int2 *__restrict__ map) {
    __shared__ __attribute__((aligned(16))) uint32_t smem[kWaves * kJT];
    const int2 e = map[blockIdx.x];
    if (st[e.x].stage != kSDom) return;  // finished early (device-side error)
    item_dom<M>(inst[e.x], e.y, smem);
}

// Parked instances -> first peeling level (the level-0 split of every point).
__global__ void k_engine_resume(const EInst *__restrict__ inst, EState *st, int32_t b0, int32_t nb,
                                EGlobal *g) {
    const int32_t q = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
    if (q >= nb) return;  // g was cleared by the reset kernel
    const int32_t b = b0 + q;
    const EInst &I = inst[b];
    EState &S = st[b];
    EScal *sc = at<EScal>(I.ws, I.L.scal);
    if (S.stage != kSDom || sc->err != 0) {  // already done: counts as finished
        S.stage = kSDone;
        S.word = 0ull;
        atomicAdd(&g->finished, 1u);
        return;
    }
    sc->n_before = 0;
    sc->last_front = -1;
    sc->rank2_overflow = 0;
    S.arg = 0;
    S.n = I.N;
    S.p0 = S.p1 = 0;
    S.done = 0;
    if (I.M == 2) {
        S.stage = kSRank2;
        S.word = 1ull;
    } else if (I.N <= kESplitOne) {
        S.stage = kSSplit1;
        S.word = 1ull;
    } else {
        S.stage = kSSplitC;
        S.word = (uint64_t)cdiv(I.N, kESplit);
    }
}

}  // namespace

hipError_t engine_dom_launch(int M, const EInst *inst, const EState *st, const int2 *map,
                             int64_t nblocks, hipStream_t s) {
    if (nblocks <= 0) return hipSuccess;
    switch (M) {
#define NSGA3_CASE(m)                                                                              \
    case m:                                                                                        \
        hipLaunchKernelGGL(k_engine_dom<m>, dim3((unsigned)nblocks), dim3(kEThreads), 0, s, inst, \
                           st, map);                                                               \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t engine_resume(const EInst *inst, EState *st, int32_t b0, int32_t nb, EGlobal *g,
                         hipStream_t s) {
    hipLaunchKernelGGL(k_engine_resume, dim3((unsigned)cdiv(nb, 64)), dim3(64), 0, s, inst, st, b0,
                       nb, g);
    return hipGetLastError();
}

hipError_t engine_init(const EInst *inst, EState *st, EGlobal *g, int32_t B, int32_t nclass,
                       hipStream_t s) {
    const int32_t n = B > nclass ? B : nclass;
    hipLaunchKernelGGL(k_engine_init, dim3((unsigned)cdiv(n, 64)), dim3(64), 0, s, inst, st, g, B,
                       nclass);
    return hipGetLastError();
}

hipError_t engine_launch(int M, const EInst *inst, EState *st, int32_t b0, int32_t nb, EGlobal *g,
                         EStats *stats, int32_t stop_stage, int grid, hipStream_t s) {
    switch (M) {
#define NSGA3_CASE(m)                                                                              \
    case m:                                                                                        \
        hipLaunchKernelGGL(k_engine<m>, dim3((unsigned)grid), dim3(kEThreads), 0, s, inst, st, b0, \
                           nb, g, stats, stop_stage);                                              \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int engine_blocks_per_cu(int M) {
    int nb = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (M) {
#define NSGA3_OCC(m) case m: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_engine<m>, kEThreads, 0); break;
        NSGA3_OCC(2) NSGA3_OCC(3) NSGA3_OCC(4) NSGA3_OCC(5) NSGA3_OCC(6) NSGA3_OCC(7) NSGA3_OCC(8)
        NSGA3_OCC(9) NSGA3_OCC(10) NSGA3_OCC(11) NSGA3_OCC(12) NSGA3_OCC(13) NSGA3_OCC(14)
        NSGA3_OCC(15) NSGA3_OCC(16)
#undef NSGA3_OCC
        default: return 0;
    }
    return e == hipSuccess ? nb : 0;
}

}  // namespace nsga3
