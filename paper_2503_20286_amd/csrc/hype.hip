// Environmental selection of TensorHypE (Sec. IV-C; Supplementary Alg. S.10,
// S.11): after the nondominated sort of the merged population (ranks r and
// the last admitted front l for a population of n), the members of F_l with
// the largest Monte Carlo hypervolume estimates fill the places left.
//
//   k = |{r <= l}| - n;  alpha_c = (1/c) prod_{i=1}^{c-1} (k - i) / (N - i)
//   f_l = the per-objective minimum over all N points, f_u = the reference
//   point, V = prod_j (f_u,j - f_l,j); sample i is S_i = f_l + U_i (f_u - f_l)
//   (U the caller's uniform draws, each sample rounded to float32 once);
//   count_i = #{p : F_p <= S_i}; HV_p = sum over the samples i that F_p
//   weakly dominates with count_i <= k of alpha_{count_i}, times V / s.
//
//  k_hv_samples  sample order keys, V, and the draws' finiteness
//  k_hv_counts   count_i: each lane probes the block tables of all points
//                (built by the dominance stage) with its samples: the members
//                with every key <= the sample's are one AND of prefix masks
//  k_hv_alpha    the alpha weights: chunked products in one work-group
//  k_hv_weights  w_i = alpha_{count_i} for 1 <= count_i <= k (else 0), and the
//                flags of those samples (compacted in order afterwards)
//  k_hv_sum      per point of r <= l: the weights of the kept samples it
//                dominates, added in sample order in float64 (the order of the
//                oracle's sum), staged through LDS
//  k_hv_keys     sort keys: F_l members by descending estimate (then index),
//                everything else after them; flags of r < l
//  k_hv_pick     the first R of the sorted order join the selection
#include <float.h>

#include "bitdom.h"
#include "kernels.h"
#include "prims.h"

namespace nsga3 {

constexpr int kHvThreads = 256;
constexpr int kHvSumChunk = 512;       // samples staged per step of k_hv_sum

struct HvState {
    double V;                           // box volume prod (f_u - f_l)
    int64_t k;                          // |S| - n
    uint32_t nrel;                      // samples with 1 <= count <= k
};

__global__ void k_hv_samples(const float *__restrict__ U, int64_t s, int M, const float *__restrict__ vref,
                             DevScalars *sc, uint32_t *__restrict__ skeys, HvState *hs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) {
        double V = 1.0;
        bool ok = true;
        for (int j = 0; j < M; ++j) {
            ok = ok && isfinite(vref[j]);
            V = V * ((double)vref[j] - (double)key_to_float(sc->min_key[j]));
        }
        hs->V = V;
        if (!ok) atomicOr(&sc->err, kErrNonfiniteObj);
    }
    if (t >= s * M) return;
    const int j = (int)(t % M);
    const float u = U[t];
    if (!isfinite(u)) atomicOr(&sc->err, kErrNonfiniteObj);
    const double fl = (double)key_to_float(sc->min_key[j]);
    const float x = (float)(fl + (double)u * ((double)vref[j] - fl));
    skeys[t] = order_key(x);
}

// count_i over all points: work-group (tile group jg of kHvTiles x 512
// samples, chunk group cg of kHvChunks table chunks), one atomic per sample.
constexpr int kHvTiles = 2;
constexpr int kHvChunks = 2;

template <int M>
__global__ __launch_bounds__(kFwdThreads) void k_hv_counts(const uint32_t *__restrict__ tabs,
                                                           int32_t nblk,
                                                           const uint32_t *__restrict__ skeys,
                                                           int64_t s, int32_t *__restrict__ count,
                                                           const DevScalars *__restrict__ sc) {
    constexpr int CB = count_chunk<M>();
    constexpr int TS = blk_stride(M);
    __shared__ __attribute__((aligned(16))) uint32_t lt[CB * TS];
    if (sc->err) return;
    const int32_t nIC = (nblk + CB - 1) / CB;
    const int32_t c0 = (int32_t)blockIdx.y * kHvChunks;
    const int32_t c1 = min(c0 + kHvChunks, nIC);
    if (c0 >= nIC) return;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const int lane = (int)lane_id();
    uint32_t x[kHvTiles][kTJ][M];
    int32_t cnt[kHvTiles][kTJ];
#pragma unroll
    for (int t = 0; t < kHvTiles; ++t)
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int64_t i = ((int64_t)blockIdx.x * kHvTiles + t) * kTileJ + w * kWave * kTJ + u * kWave + lane;
            cnt[t][u] = 0;
#pragma unroll
            for (int k = 0; k < M; ++k) x[t][u][k] = i < s ? skeys[i * M + k] : 0u;  // 0: below every key
        }
    for (int32_t c = c0; c < c1; ++c) {
        const int32_t b0 = c * CB;
        const int32_t nb = min(CB, nblk - b0);
        __syncthreads();
        stage_tables<M>(lt, tabs, b0, nb);
        __syncthreads();
        for (int32_t b = 0; b < nb; ++b) {
            const uint32_t *T = lt + b * TS;
#pragma unroll
            for (int t = 0; t < kHvTiles; ++t) {
                int ko[kTJ * M];
                uint32_t xx[kTJ * M];
                uint64_t pm[kTJ * M];
#pragma unroll
                for (int u = 0; u < kTJ; ++u)
#pragma unroll
                    for (int k = 0; k < M; ++k) {
                        ko[u * M + k] = k;
                        xx[u * M + k] = x[t][u][k];
                    }
                masks_many64<M, kTJ * M, true>(T, ko, xx, pm);
#pragma unroll
                for (int u = 0; u < kTJ; ++u) {
                    uint64_t m = ~0ull;
#pragma unroll
                    for (int k = 0; k < M; ++k) m &= pm[u * M + k];
                    cnt[t][u] += __popcll(m);
                }
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kHvTiles; ++t)
#pragma unroll
        for (int u = 0; u < kTJ; ++u) {
            const int64_t i = ((int64_t)blockIdx.x * kHvTiles + t) * kTileJ + w * kWave * kTJ + u * kWave + lane;
            if (i < s && cnt[t][u]) atomicAdd(&count[i], cnt[t][u]);
        }
}

// alpha_c = prod_{i<c} f_i / c with f_i = (k - i) / (N - i): thread q multiplies
// the factors of its chunk of c, a scan multiplies the chunk products, and each
// c is its chunk's prefix times its own running product.
__global__ __launch_bounds__(1024) void k_hv_alpha(int64_t N, int64_t n, const DevScalars *__restrict__ sc,
                                                   double *__restrict__ alpha, HvState *hs) {
    __shared__ double part[1024];
    if (sc->err) return;
    const int64_t k = sc->n_before + (int64_t)sc->last_front_size - n;
    if (threadIdx.x == 0) hs->k = k;
    if (k <= 0) return;
    const int64_t per = (k + blockDim.x - 1) / blockDim.x;
    const int64_t c0 = 1 + (int64_t)threadIdx.x * per;
    const int64_t c1 = c0 + per <= k + 1 ? c0 + per : k + 1;
    double p = 1.0;
    for (int64_t c = c0; c < c1; ++c)
        if (c > 1) p = p * ((double)(k - (c - 1)) / (double)(N - (c - 1)));
    part[threadIdx.x] = p;
    __syncthreads();
    if (threadIdx.x == 0) {  // exclusive product scan (1024 steps, one thread)
        double run = 1.0;
        for (unsigned q = 0; q < blockDim.x; ++q) {
            const double v = part[q];
            part[q] = run;
            run = run * v;
        }
    }
    __syncthreads();
    double q = part[threadIdx.x];
    for (int64_t c = c0; c < c1; ++c) {
        if (c > 1) q = q * ((double)(k - (c - 1)) / (double)(N - (c - 1)));
        alpha[c - 1] = q / (double)c;
    }
}

__global__ void k_hv_weights(int64_t s, const int32_t *__restrict__ count, const double *__restrict__ alpha,
                             double *__restrict__ w, uint8_t *__restrict__ flag,
                             const HvState *__restrict__ hs, const DevScalars *__restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= s) return;
    const int64_t c = count[i];
    const bool keep = !sc->err && c >= 1 && c <= hs->k;
    w[i] = keep ? alpha[c - 1] : 0.0;
    flag[i] = keep ? 1 : 0;
}

template <int M>
__global__ __launch_bounds__(kHvThreads) void k_hv_sum(const float *__restrict__ objs, int64_t N,
                                                        const int32_t *__restrict__ rank,
                                                        const uint32_t *__restrict__ skeys,
                                                        const double *__restrict__ w,
                                                        const int32_t *__restrict__ rel, int64_t s,
                                                        const HvState *__restrict__ hs,
                                                        const DevScalars *__restrict__ sc,
                                                        double *__restrict__ d) {
    __shared__ uint32_t ks[M][kHvSumChunk];
    __shared__ double ws[kHvSumChunk];
    if (sc->err) return;
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t l = sc->last_front;
    const bool mine = p < N && rank[p] <= l;
    uint32_t key[M];
#pragma unroll
    for (int k = 0; k < M; ++k) key[k] = p < N ? order_key(objs[p * M + k]) : 0xffffffffu;
    const uint32_t nrel = hs->nrel;
    double acc = 0.0;
    for (uint32_t q0 = 0; q0 < nrel; q0 += kHvSumChunk) {
        const uint32_t nq = nrel - q0 < (uint32_t)kHvSumChunk ? nrel - q0 : (uint32_t)kHvSumChunk;
        __syncthreads();
        for (uint32_t q = threadIdx.x; q < nq; q += blockDim.x) {
            const int32_t i = rel[q0 + q];
#pragma unroll
            for (int k = 0; k < M; ++k) ks[k][q] = skeys[(int64_t)i * M + k];
            ws[q] = w[i];
        }
        __syncthreads();
        if (mine) {
            for (uint32_t q = 0; q < nq; ++q) {
                bool dom = true;
#pragma unroll
                for (int k = 0; k < M; ++k) dom = dom && key[k] <= ks[k][q];
                acc = acc + (dom ? ws[q] : 0.0);
            }
        }
    }
    if (p < N) d[p] = mine ? acc * hs->V / (double)s : -INFINITY;
}

// Sort keys of the selection: members of F_l by descending estimate (the
// estimate is >= 0, so its bits order like it), ties in index order (the sort
// is stable and starts in index order); every other point after them.
__global__ void k_hv_keys(int64_t N, const int32_t *__restrict__ rank, const double *__restrict__ d,
                          uint64_t *__restrict__ key, uint32_t *__restrict__ val,
                          uint8_t *__restrict__ selflag, const DevScalars *__restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t l = sc->last_front;
    const int32_t r = rank[i];
    key[i] = r == l ? 0x7fffffffffffffffull - (uint64_t)__double_as_longlong(d[i]) : ~0ull;
    val[i] = (uint32_t)i;
    selflag[i] = r < l ? 1 : 0;
}

__global__ void k_hv_pick(const uint32_t *__restrict__ val, uint8_t *__restrict__ selflag,
                          const DevScalars *__restrict__ sc) {
    if (sc->err) return;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < sc->num_from_last) selflag[val[q]] = 1;
}

__global__ void k_hv_zero(int32_t *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t hype_extra_bytes(int64_t N, int M, int64_t s) {
    return up256(sizeof(HvState)) + up256(4 * (size_t)s * M) + up256(4 * (size_t)s) +
           up256(8 * (size_t)s) + up256((size_t)s) + up256(4 * (size_t)s) + up256(8 * (size_t)N) +
           up256(8 * (size_t)N) + up256(compact_temp_bytes(s));
}

hipError_t run_hype(const HypeViews &v, hipStream_t st) {
    char *w = (char *)v.extra;
    HvState *hs = (HvState *)w;
    w += up256(sizeof(HvState));
    uint32_t *skeys = (uint32_t *)w;
    w += up256(4 * (size_t)v.s * v.M);
    int32_t *count = (int32_t *)w;
    w += up256(4 * (size_t)v.s);
    double *wt = (double *)w;
    w += up256(8 * (size_t)v.s);
    uint8_t *flag = (uint8_t *)w;
    w += up256((size_t)v.s);
    int32_t *rel = (int32_t *)w;
    w += up256(4 * (size_t)v.s);
    double *alpha = (double *)w;
    w += up256(8 * (size_t)v.N);
    double *dd = v.d ? v.d : (double *)w;
    w += up256(8 * (size_t)v.N);
    uint32_t *ctemp = (uint32_t *)w;
    const int64_t N = v.N, s = v.s;
    const int M = v.M;
    hipLaunchKernelGGL(k_hv_zero, dim3((unsigned)((s + 255) / 256 < 2048 ? (s + 255) / 256 : 2048)),
                       dim3(256), 0, st, count, s);
    const int64_t sm = s * M;
    hipLaunchKernelGGL(k_hv_samples, dim3((unsigned)((sm + 255) / 256)), dim3(256), 0, st, v.U, s, M,
                       v.vref, v.sc, skeys, hs);
    const int32_t nblk = (int32_t)((N + kBlk - 1) / kBlk);
    const unsigned nTG = (unsigned)((s + (int64_t)kHvTiles * kTileJ - 1) / ((int64_t)kHvTiles * kTileJ));
    hipError_t e = hipSuccess;
    switch (M) {
#define NSGA3_CASE(m)                                                                               \
    case m: {                                                                                       \
        const int32_t nIC = (nblk + count_chunk<m>() - 1) / count_chunk<m>();                      \
        const unsigned nCG = (unsigned)((nIC + kHvChunks - 1) / kHvChunks);                        \
        hipLaunchKernelGGL(k_hv_counts<m>, dim3(nTG, nCG), dim3(kFwdThreads), 0, st, v.tabs_all,    \
                           nblk, skeys, s, count, v.sc);                                           \
        break;                                                                                      \
    }
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_hv_alpha, dim3(1), dim3(1024), 0, st, N, v.n, v.sc, alpha, hs);
    const unsigned gS = (unsigned)((s + 255) / 256);
    hipLaunchKernelGGL(k_hv_weights, dim3(gS), dim3(256), 0, st, s, count, alpha, wt, flag, hs, v.sc);
    compact_flags(flag, s, rel, s, ctemp, &hs->nrel, st);
    const unsigned gN = (unsigned)((N + kHvThreads - 1) / kHvThreads);
    switch (M) {
#define NSGA3_CASE(m)                                                                               \
    case m:                                                                                         \
        hipLaunchKernelGGL(k_hv_sum<m>, dim3(gN), dim3(kHvThreads), 0, st, v.objs, N, v.rank,       \
                           skeys, wt, rel, s, hs, v.sc, dd);                                       \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_hv_keys, dim3(gN), dim3(kHvThreads), 0, st, N, v.rank, dd, v.skey, v.sval,
                       v.selflag, v.sc);
    bool in_alt = false;
    radix_sort_pairs(v.skey, v.sval, v.skey_alt, v.sval_alt, N, 64, v.temp, st, &in_alt);
    const uint32_t *sval = in_alt ? v.sval_alt : v.sval;
    hipLaunchKernelGGL(k_hv_pick, dim3(gN), dim3(kHvThreads), 0, st, sval, v.selflag, v.sc);
    compact_flags(v.selflag, N, v.selected, v.n, v.temp, &v.sc->n_selected, st);
    if (v.info) run_finalize(v.info, v.n, v.sc, st);
    e = hipGetLastError();
    return e;
}

}  // namespace nsga3
