// Normalisation, association, niche counting and niche-preserving selection
// on gfx950 (stages after the nondominated sort).
//
//  a4/a5  Alg. S.5: ideal point z (minimum over all points, which equals the
//         minimum over S = {rank <= l}: every minimiser of an objective is
//         dominated only by other minimisers, so one of them is nondominated),
//         extreme points by the achievement scalarising function with weights
//         1 (own axis) and 1e-6 (other axes, applied as x 1e6), hyperplane
//         intercepts from E b = 1 by Gaussian elimination with partial
//         pivoting in float64, with the nadir point as fallback.
//  a6     Eq. (10): perpendicular distance of f' = (f - z) / a to every
//         reference line.  argmin_j d_ij = argmax_j f'.rhat_j (f', rhat >= 0),
//         so candidates are screened by that dot product in float32 and the
//         survivors are re-scored in float64 with the residual form
//         ||f' - (f'.rhat) rhat||.
//  a7     Eq. (11): niche counts rho over the admitted members (rank < l) and
//         the per-reference member counts of the last front (Eq. (12)).
//  a8     Alg. S.1 inner loop, evaluated in parallel: last-front member i of
//         reference j gets the level rho_j + t_i, t_i its position among the
//         members of j ordered by (distance, index); the loop picks exactly the
//         R smallest (level, reference) pairs, found by a threshold search.
//  a9     Eq. (13): ascending indices of the selected points.
#include <float.h>

#include "kernels.h"
#include "prims.h"
#include "stage_math.h"

namespace nsga3 {

constexpr int kNormThreads = 256;
constexpr int kRankGroup = 256;                   // threads of a bucket-rank work-group
constexpr int kRankSplit = 4;                     // threads sharing one member's count
constexpr int kRankMembers = kRankGroup / kRankSplit;  // members ranked per work-group
constexpr int kNormBlocksMax = 256;

// ---------------------------------------------------------------------------
// init: clear per-call scalars and counters (fill kernels, no memset nodes)
// ---------------------------------------------------------------------------
__global__ void k_init_scalars(DevScalars *sc) {
    const int t = threadIdx.x;
    if (t == 0) {
        sc->err = 0;
        sc->last_front = 0;
        sc->num_fronts = 0;
        sc->last_front_size = 0;
        sc->n_before = 0;
        sc->num_from_last = 0;
        sc->fallback = 0;
        sc->near_ties = 0;
        sc->nf = sc->nu = 0;
        sc->bar_count = 0;
        sc->bar_gen = 0;
        sc->level_V = 0;
        sc->ref_thr = 0;
    }
    if (t < 16) {
        sc->min_key[t] = 0xffffffffu;
        sc->a[t] = 1.0;
        sc->z[t] = 0.0;
    }
}

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

hipError_t run_init(DevScalars *sc, int32_t *zero_i32[], const int64_t zero_n[], int nzero,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_init_scalars, dim3(1), dim3(64), 0, s, sc);
    for (int q = 0; q < nzero; ++q) {
        if (!zero_i32[q] || zero_n[q] <= 0) continue;
        int64_t nb = (zero_n[q] + 255) / 256;
        if (nb > 2048) nb = 2048;
        hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)nb), dim3(256), 0, s, zero_i32[q], zero_n[q], 0);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// reference directions: validity and unit vectors (float64 and float32)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint16_t bf16_rne(float f) {
    const uint32_t u = __float_as_uint(f);
    return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);  // finite inputs only
}

// Unit reference directions in float64 and float32, and in bfloat16 for the
// matrix-core screening: [Hpad x KP] (KP = 8 for M <= 8, else 16), rows and
// columns beyond (H, M) zero.
__global__ void k_refs(const float *__restrict__ refs, int H, int M, double *__restrict__ rhat64,
                       float *__restrict__ rhat32, uint16_t *__restrict__ rhat16, int Hpad, int KP,
                       DevScalars *__restrict__ sc) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < Hpad && rhat16) {
        for (int k = 0; k < KP; ++k) rhat16[(int64_t)j * KP + k] = 0;
    }
    if (j >= H) return;
    if (!unit_reference(refs, j, M, rhat64, rhat32)) {
        atomicOr(&sc->err, (uint32_t)kErrBadRef);
        return;
    }
    if (rhat16)
        for (int k = 0; k < M; ++k) rhat16[(int64_t)j * KP + k] = bf16_rne(rhat32[(int64_t)j * M + k]);
}

__device__ __forceinline__ double ideal(const DevScalars *sc, int k) {
    return (double)key_to_float(sc->min_key[k]);
}

// ---------------------------------------------------------------------------
// a4: extreme-point partials per block (ASF argmin per axis) and nadir partials
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kNormThreads) void k_extreme_partial(
    const float *__restrict__ objs, int64_t N, int M, const int32_t *__restrict__ rank,
    const DevScalars *__restrict__ sc, double *__restrict__ p_asf, int32_t *__restrict__ p_idx,
    double *__restrict__ p_nad) {
    __shared__ double s_asf[kNormThreads / kWave][16];
    __shared__ int32_t s_idx[kNormThreads / kWave][16];
    __shared__ double s_nad[kNormThreads / kWave][16];
    if (sc->err) return;
    const int32_t l = sc->last_front;
    double z[16], best[16], nad[16];
    int32_t bidx[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        z[k] = k < M ? ideal(sc, k) : 0.0;
        best[k] = DBL_MAX;
        bidx[k] = 0x7fffffff;
        nad[k] = 0.0;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += stride) {
        if (rank[i] > l) continue;
        double g[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) g[k] = k < M ? (double)objs[i * M + k] - z[k] : 0.0;
        asf_fold<16>(g, M, (int32_t)i, best, bidx, nad);
    }
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j >= M) continue;
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
        if (lane_id() == 0) { s_asf[w][j] = b; s_idx[w][j] = bi; s_nad[w][j] = nd; }
    }
    __syncthreads();
    if ((int)threadIdx.x < M) {
        const int j = threadIdx.x;
        double b = s_asf[0][j];
        int32_t bi = s_idx[0][j];
        double nd = s_nad[0][j];
        for (int q = 1; q < kNormThreads / kWave; ++q) {
            if (s_asf[q][j] < b || (s_asf[q][j] == b && s_idx[q][j] < bi)) { b = s_asf[q][j]; bi = s_idx[q][j]; }
            nd = s_nad[q][j] > nd ? s_nad[q][j] : nd;
        }
        p_asf[blockIdx.x * M + j] = b;
        p_idx[blockIdx.x * M + j] = bi;
        p_nad[blockIdx.x * M + j] = nd;
    }
}

// ---------------------------------------------------------------------------
// a5: reduce the partials, build E, solve E b = 1, intercepts / fallback.
// One block of kSolveThreads: every thread folds its share of the partials
// for all axes, the waves fold across lanes, wave 0 across waves.
// ---------------------------------------------------------------------------
constexpr int kSolveThreads = 1024;

template <int M>
__global__ __launch_bounds__(kSolveThreads) void k_solve(const float *__restrict__ objs, int nparts,
                                                         const double *__restrict__ p_asf,
                                                         const int32_t *__restrict__ p_idx,
                                                         const double *__restrict__ p_nad,
                                                         DevScalars *__restrict__ sc) {
    constexpr int kW = kSolveThreads / kWave;
    __shared__ double w_asf[kW][16], w_nad[kW][16];
    __shared__ int32_t w_idx[kW][16];
    __shared__ int32_t s_e[16];
    __shared__ double s_nadir[16];
    if (sc->err) return;
    const int lane = (int)lane_id(), wid = (int)threadIdx.x / kWave;
    for (int j = 0; j < M; ++j) {
        double b = DBL_MAX;
        int32_t bi = 0x7fffffff;
        double nd = 0.0;
        for (int q = threadIdx.x; q < nparts; q += kSolveThreads) {
            const double a = p_asf[q * M + j];
            const int32_t ai = p_idx[q * M + j];
            if (a < b || (a == b && ai < bi)) { b = a; bi = ai; }
            const double n = p_nad[q * M + j];
            nd = n > nd ? n : nd;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(b, o, 64);
            const int32_t oi = __shfl_xor(bi, o, 64);
            if (ob < b || (ob == b && oi < bi)) { b = ob; bi = oi; }
            const double on = __shfl_xor(nd, o, 64);
            nd = on > nd ? on : nd;
        }
        if (lane == 0) { w_asf[wid][j] = b; w_idx[wid][j] = bi; w_nad[wid][j] = nd; }
    }
    __syncthreads();
    if (wid != 0) return;
    for (int j = 0; j < M; ++j) {
        double b = lane < kW ? w_asf[lane][j] : DBL_MAX;
        int32_t bi = lane < kW ? w_idx[lane][j] : 0x7fffffff;
        double nd = lane < kW ? w_nad[lane][j] : 0.0;
        for (int o = 32; o > 0; o >>= 1) {
            const double ob = __shfl_xor(b, o, 64);
            const int32_t oi = __shfl_xor(bi, o, 64);
            if (ob < b || (ob == b && oi < bi)) { b = ob; bi = oi; }
            const double on = __shfl_xor(nd, o, 64);
            nd = on > nd ? on : nd;
        }
        if (lane == 0) { s_e[j] = bi; s_nadir[j] = nd; }
    }
    double z[M], a[M];
#pragma unroll
    for (int k = 0; k < M; ++k) z[k] = ideal(sc, k);
    const int fb = solve_intercepts_wave<M>(objs, s_e, s_nadir, z, a);
    if (lane != 0) return;
    for (int k = 0; k < M; ++k) {
        sc->z[k] = z[k];
        sc->a[k] = a[k];
    }
    sc->fallback = fb;
}

// ---------------------------------------------------------------------------
// a6/a7: association (float32 screening, float64 re-scoring) and counts.
// The reference loop is uniform, so the float32 unit references stream
// through scalar loads.
// ---------------------------------------------------------------------------
template <int M>
__global__ __launch_bounds__(kNormThreads) void k_associate(
    const float *__restrict__ objs, int64_t N, const int32_t *__restrict__ rank,
    const double *__restrict__ rhat64, const float *__restrict__ rhat32, int H,
    int32_t *__restrict__ niche, float *__restrict__ dist, double *__restrict__ dist64,
    int32_t *__restrict__ rho, int32_t *__restrict__ bcount, uint8_t *__restrict__ selflag,
    DevScalars *__restrict__ sc) {
    __shared__ int32_t hist[2 * kLdsNicheRefs];
    if (sc->err) return;
    const float *__restrict__ R = rhat32;  // uniform reads: scalar loads
    const int32_t l = sc->last_front;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int32_t r = i < N ? rank[i] : 0x7fffffff;
    int cls = -1;
    int32_t best = 0;
    if (r <= l) {
        double fp[M];
        float y[M];
        const float l1 = normalise_point<M>(objs + i * M, sc->z, sc->a, fp, y);
        double d1, d2;
        associate_point<M>(fp, y, l1, R, rhat64, H, best, d1, d2);
        niche[i] = best;
        if (dist) dist[i] = (float)d1;
        dist64[i] = d1;
        if (near_tie(d1, d2)) atomicAdd(&sc->near_ties, 1);
        cls = r < l ? 0 : 1;
        selflag[i] = r < l ? 1 : 0;
    } else if (i < N) {
        niche[i] = -1;
        if (dist) dist[i] = -1.0f;
        dist64[i] = -1.0;
        selflag[i] = 0;
    }
    niche_count_block(H, cls, best, rho, bcount, hist);
}

// ---------------------------------------------------------------------------
// a6/a7, matrix-core form: the screening dot products s = y . rhat are one
// bfloat16 MFMA per 32 references x 32 points (float32 accumulate); refs are
// the A operand (rows), points the B operand (columns), so each lane holds one
// point (column l % 32) and 16 of the 32 references of the tile.  The band
// covers the bfloat16 rounding of both operands; survivors are re-scored in
// float64 exactly as in the float32 form.
// ---------------------------------------------------------------------------
typedef float mfma_f16v __attribute__((ext_vector_type(16)));
typedef short mfma_s4v __attribute__((ext_vector_type(4)));
typedef __bf16 mfma_b8v __attribute__((ext_vector_type(8)));

template <int KP>
struct BfOperand;
template <>
struct BfOperand<8> {
    using T = mfma_s4v;  // 4 bf16 per lane (k = 4 * (lane / 32) + v)
    static __device__ __forceinline__ mfma_f16v mma(T a, T b, mfma_f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void set(T &x, int v, uint16_t bits) { x[v] = (short)bits; }
    static constexpr int kPerLane = 4;
};
template <>
struct BfOperand<16> {
    using T = mfma_b8v;  // 8 bf16 per lane (k = 8 * (lane / 32) + v)
    static __device__ __forceinline__ mfma_f16v mma(T a, T b, mfma_f16v c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ void set(T &x, int v, uint16_t bits) {
        x[v] = __builtin_bit_cast(__bf16, bits);
    }
    static constexpr int kPerLane = 8;
};

template <int M>
__global__ __launch_bounds__(256) void k_associate_bf16(
    const float *__restrict__ objs, int64_t N, const int32_t *__restrict__ rank,
    const double *__restrict__ rhat64, const uint16_t *__restrict__ rhat16, int H,
    int32_t *__restrict__ niche, float *__restrict__ dist, double *__restrict__ dist64,
    int32_t *__restrict__ rho, int32_t *__restrict__ bcount, uint8_t *__restrict__ selflag,
    DevScalars *__restrict__ sc) {
    constexpr int KP = M <= 8 ? 8 : 16;
    using Op = BfOperand<KP>;
    constexpr int KL = Op::kPerLane;
    __shared__ int32_t hist[2 * kLdsNicheRefs];
    if (sc->err) return;
    const int32_t l = sc->last_front;
    const int lane = (int)lane_id();
    const int half = lane >> 5;                       // which k-slice / row half this lane holds
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t i = wave * 32 + (lane & 31);        // this lane's point (shared with lane ^ 32)
    const bool inrange = i < N;
    const int32_t r = inrange ? rank[i] : 0x7fffffff;
    const bool active = inrange && r <= l;
    double fp[M];
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        fp[k] = active ? ((double)objs[i * M + k] - sc->z[k]) / sc->a[k] : 0.0;
        mx = fp[k] > mx ? fp[k] : mx;
    }
    float y[M];
    float n2 = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        y[k] = mx > 0.0 ? (float)(fp[k] / mx) : 0.0f;
        n2 = __fmaf_rn(y[k], y[k], n2);
    }
    // B operand: this lane's point, k-slice [KL * half, KL * half + KL)
    typename Op::T bop;
#pragma unroll
    for (int v = 0; v < KL; ++v) {
        const int k = KL * half + v;
        float val = 0.0f;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (q == k) val = y[q];
        Op::set(bop, v, bf16_rne(val));
    }
    const int ntiles = (H + 31) / 32;
    float smax = -FLT_MAX;
    for (int tl = 0; tl < ntiles; ++tl) {
        const typename Op::T aop = *reinterpret_cast<const typename Op::T *>(
            rhat16 + ((int64_t)(tl * 32 + (lane & 31)) * KP + KL * half));
        mfma_f16v acc = {};
        acc = Op::mma(aop, bop, acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = tl * 32 + 8 * (v / 4) + 4 * half + (v % 4);
            if (j < H) smax = acc[v] > smax ? acc[v] : smax;
        }
    }
    smax = fmaxf(smax, __shfl_xor(smax, 32, 64));
    // |s_bf16 - s| <= (2 u + u^2) ||y||_2 + float32 rounding, u = 2^-8; doubled
    const float band = 2.0f * 1.01f * (0.0078125f + 0.000244f) * sqrtf(n2) + 1e-30f;
    const float thr = smax - band;
    double d1 = DBL_MAX, d2 = DBL_MAX;
    int32_t best = 0x7fffffff;
    for (int tl = 0; tl < ntiles; ++tl) {
        const typename Op::T aop = *reinterpret_cast<const typename Op::T *>(
            rhat16 + ((int64_t)(tl * 32 + (lane & 31)) * KP + KL * half));
        mfma_f16v acc = {};
        acc = Op::mma(aop, bop, acc);
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int j = tl * 32 + 8 * (v / 4) + 4 * half + (v % 4);
            if (j >= H || acc[v] < thr || !active) continue;
            const double d = line_distance<M>(fp, rhat64 + (int64_t)j * M);
            if (d < d1 || (d == d1 && j < best)) { d2 = d1; d1 = d; best = j; }
            else if (d < d2 || d == d2) { d2 = d < d2 ? d : d2; }
        }
    }
    // merge with the lane holding the other 16 references of every tile
    const double od1 = __shfl_xor(d1, 32, 64);
    const double od2 = __shfl_xor(d2, 32, 64);
    const int32_t obest = __shfl_xor(best, 32, 64);
    if (od1 < d1 || (od1 == d1 && obest < best)) {
        d2 = fmin(d1, od2);
        d1 = od1;
        best = obest;
    } else {
        d2 = fmin(d2, od1);
    }
    int cls = -1;
    if (inrange && half == 0) {
        if (!active) {
            niche[i] = -1;
            if (dist) dist[i] = -1.0f;
            dist64[i] = -1.0;
            selflag[i] = 0;
        } else {
            niche[i] = best;
            if (dist) dist[i] = (float)d1;
            dist64[i] = d1;
            if (near_tie(d1, d2)) atomicAdd(&sc->near_ties, 1);
            cls = r < l ? 0 : 1;
            selflag[i] = r < l ? 1 : 0;
        }
    }
    niche_count_block(H, cls, best, rho, bcount, hist);
}

// ---------------------------------------------------------------------------
// a8 plan: bucket offsets of the last front by reference, and the selection
// threshold.  For threshold V, C(V) = sum_j clamp(V - rho_j, 0, b_j) members
// have level < V.  V* = max{V : C(V) <= R}; the remaining R - C(V*) picks are
// the level-V* members of the lowest-indexed references.  One block.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(1024) void k_niche_plan(int H, const int32_t *__restrict__ rho,
                                                     const int32_t *__restrict__ bcount,
                                                     int32_t *__restrict__ bstart,
                                                     int32_t *__restrict__ bcursor,
                                                     int32_t *__restrict__ gstart,
                                                     DevScalars *__restrict__ sc) {
    __shared__ uint32_t lds[17];
    __shared__ int64_t red[16];
    __shared__ int64_t s_vmax;
    if (sc->err) return;
    const int64_t R = sc->num_from_last;
    // bucket starts (exclusive scan of bcount), chunked by blockDim
    uint32_t run = 0, grun = 0;
    int64_t vmax = 0;
    for (int base = 0; base < H; base += blockDim.x) {
        const int j = base + threadIdx.x;
        const uint32_t v = j < H ? (uint32_t)bcount[j] : 0u;
        if (j < H) {
            const int64_t top = (int64_t)rho[j] + bcount[j];
            vmax = top > vmax ? top : vmax;
        }
        uint32_t tot, gtot;
        const uint32_t ex = block_exclusive_scan(v, lds, &tot);
        const uint32_t gex = block_exclusive_scan((v + kRankMembers - 1) / kRankMembers, lds, &gtot);
        if (j < H) {
            bstart[j] = (int32_t)(run + ex);
            bcursor[j] = (int32_t)(run + ex);
            gstart[j] = (int32_t)(grun + gex);
        }
        run += tot;
        grun += gtot;
    }
    if (threadIdx.x == 0) {
        bstart[H] = (int32_t)run;
        gstart[H] = (int32_t)grun;
    }
    vmax = wave_max(vmax);
    if (lane_id() == 0) red[threadIdx.x / kWave] = vmax;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t m = 0;
        for (unsigned q = 0; q < blockDim.x / kWave; ++q) m = red[q] > m ? red[q] : m;
        s_vmax = m;
    }
    __syncthreads();
    // binary search for V* in [0, vmax]: C is non-decreasing, C(0) = 0 <= R;
    // the counts are read from LDS when they fit (one global read each, not
    // one per search step)
    constexpr int kLdsRefs = 4096;
    __shared__ int32_t s_rho[kLdsRefs], s_bc[kLdsRefs];
    const int32_t *rho_r = rho, *bc_r = bcount;
    if (H <= kLdsRefs) {
        for (int j = threadIdx.x; j < H; j += blockDim.x) {
            s_rho[j] = rho[j];
            s_bc[j] = bcount[j];
        }
        __syncthreads();
        rho_r = s_rho;
        bc_r = s_bc;
    }
    // (one wave searches: no block barriers inside the loop)
    __shared__ int64_t s_V;
    if (threadIdx.x < kWave) {
        int64_t lo = 0, hi = s_vmax;
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) >> 1;
            int64_t c = 0;
            for (int j = threadIdx.x; j < H; j += kWave) {
                int64_t t = mid - rho_r[j];
                t = t < 0 ? 0 : t;
                c += t < bc_r[j] ? t : bc_r[j];
            }
            c = wave_sum(c);
            if (c <= R) lo = mid; else hi = mid - 1;
        }
        if (threadIdx.x == 0) s_V = lo;
    }
    __syncthreads();
    const int64_t V = s_V;
    int64_t cV = 0;
    for (int j = threadIdx.x; j < H; j += blockDim.x) {
        int64_t t = V - rho[j];
        t = t < 0 ? 0 : t;
        cV += t < bcount[j] ? t : bcount[j];
    }
    cV = wave_sum(cV);
    __syncthreads();
    if (lane_id() == 0) red[threadIdx.x / kWave] = cV;
    __syncthreads();
    int64_t CV = 0;
    for (unsigned q = 0; q < blockDim.x / kWave; ++q) CV += red[q];
    const int64_t rem = R - CV;  // picks at level V, lowest references first
    // reference threshold: the rem-th reference (ascending) with a member at level V
    int32_t thr = 0;
    uint32_t seen = 0;
    __shared__ int32_t s_thr;
    if (threadIdx.x == 0) s_thr = (rem <= 0) ? 0 : H;
    __syncthreads();
    if (rem > 0) {
        for (int base = 0; base < H; base += blockDim.x) {
            const int j = base + threadIdx.x;
            const uint32_t has = (j < H && rho[j] <= V && V < (int64_t)rho[j] + bcount[j]) ? 1u : 0u;
            uint32_t tot;
            const uint32_t ex = block_exclusive_scan(has, lds, &tot);
            if (has && (int64_t)(seen + ex) == rem - 1) s_thr = j + 1;
            seen += tot;
            __syncthreads();
            if ((int64_t)seen >= rem) break;
        }
    }
    __syncthreads();
    thr = s_thr;
    if (threadIdx.x == 0) {
        sc->level_V = (int32_t)V;
        sc->ref_thr = thr;
    }
}

// last-front members -> reference buckets (order inside a bucket is arbitrary)
__global__ __launch_bounds__(256) void k_bucket_scatter(int64_t N, int H,
                                                        const int32_t *__restrict__ rank,
                                                        const int32_t *__restrict__ niche,
                                                        const double *__restrict__ dist64,
                                                        int32_t *__restrict__ bcursor,
                                                        double *__restrict__ bd,
                                                        int32_t *__restrict__ bi,
                                                        const DevScalars *__restrict__ sc) {
    __shared__ int32_t cnt[kLdsNicheRefs];
    if (sc->err) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool member = i < N && rank[i] == sc->last_front;
    const int32_t b = member ? niche[i] : 0;
    const int32_t slot = bucket_slot_block(H, member, b, bcursor, cnt);
    if (!member) return;
    bd[slot] = dist64[i];
    bi[slot] = (int32_t)i;
}

// t_i = #members of the same reference with smaller (distance, index); pick
// when (rho + t, reference) is below the threshold.  Work-group g ranks
// kRankMembers members of one bucket (gstart maps groups to buckets) against
// the whole bucket, staged through LDS; kRankSplit adjacent lanes share a
// member, each counting every kRankSplit-th bucket entry.
__global__ __launch_bounds__(kRankGroup) void k_bucket_rank(int H, const int32_t *__restrict__ rho,
                                                            const int32_t *__restrict__ bstart,
                                                            const int32_t *__restrict__ gstart,
                                                            const double *__restrict__ bd,
                                                            const int32_t *__restrict__ bi,
                                                            uint8_t *__restrict__ selflag,
                                                            const DevScalars *__restrict__ sc) {
    constexpr int kChunk = 2048;
    __shared__ double sd[kChunk];
    __shared__ int32_t si[kChunk];
    if (sc->err) return;
    const int32_t g = blockIdx.x;
    if (g >= gstart[H]) return;
    int32_t lo = 0, hi = H - 1;  // the bucket j with gstart[j] <= g < gstart[j + 1]
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (gstart[mid] <= g) lo = mid; else hi = mid - 1;
    }
    const int32_t j = lo;
    const int32_t b0 = bstart[j], b1 = bstart[j + 1];
    const int32_t s = b0 + (g - gstart[j]) * kRankMembers + (int32_t)threadIdx.x / kRankSplit;
    const int32_t sub = (int32_t)threadIdx.x % kRankSplit;
    const bool mine = s < b1;
    const double d = mine ? bd[s] : 0.0;
    const int32_t i = mine ? bi[s] : 0;
    int32_t t = 0;
    for (int32_t c0 = b0; c0 < b1; c0 += kChunk) {
        const int32_t c1 = min(c0 + kChunk, b1);
        __syncthreads();
        for (int32_t q = c0 + (int32_t)threadIdx.x; q < c1; q += kRankGroup) {
            sd[q - c0] = bd[q];
            si[q - c0] = bi[q];
        }
        __syncthreads();
        if (mine) {
            const int32_t n = c1 - c0;
#pragma unroll 4
            for (int32_t m = sub; m < n; m += kRankSplit)
                t += (sd[m] < d || (sd[m] == d && si[m] < i)) ? 1 : 0;
        }
    }
    for (int o = 1; o < kRankSplit; o <<= 1) t += __shfl_xor(t, o, 64);  // the member's lanes
    if (!mine || sub != 0) return;
    const int64_t lev = (int64_t)rho[j] + t;
    const int64_t V = sc->level_V;
    if (lev < V || (lev == V && j < sc->ref_thr)) selflag[i] = 1;
}

__global__ void k_finalize(nsga3_info *info, int64_t K, const DevScalars *__restrict__ sc) {
    if (threadIdx.x != 0) return;
    uint32_t e = sc->err;
    if (e == 0 && (int64_t)sc->n_selected != K) e |= kErrInternal;
    nsga3_info v;
    v.status = e == 0 ? NSGA3_OK
               : (e & (kErrNonfiniteObj | kErrBadRef)) ? NSGA3_E_NONFINITE
                                                       : NSGA3_E_HIP;
    v.last_front = sc->last_front;
    v.num_fronts = sc->num_fronts;
    v.last_front_size = sc->last_front_size;
    v.num_from_last = (int32_t)sc->num_from_last;
    v.intercept_fallback = sc->fallback;
    v.near_ties = sc->near_ties;
    v.reserved = (int32_t)e;
    *info = v;
}

// ---------------------------------------------------------------------------
// One-shot niche selection (Sec. IV-A.5; the niche-selection steps of
// Alg. S.4 and the Update-Rank of Alg. S.6): instead of admitting last-front
// members one at a time, every reference with no admitted member (rho_j = 0)
// that has last-front members admits its closest one (distance, then index)
// at once.  With |E| such picks and R places left, a shortfall R > |E| is
// filled with the R - |E| lowest-index unpicked last-front members, a surplus
// keeps the R lowest-index picks.  On the shuffled population the paper
// takes as input, index order is a random order, so both fill rules are the
// random choices the algorithm makes.
// selflag values on entry: 1 admitted (rank < l), 0 otherwise; the picks are
// marked 2 by k_oneshot_pick, and k_oneshot_apply leaves 0 / 1 everywhere.
// ---------------------------------------------------------------------------
constexpr int kOsTile = 2048;   // indices per count / apply work-group (8 x 256)

// One wave per reference: the closest member of an empty niche's bucket.
__global__ __launch_bounds__(256) void k_oneshot_pick(int H, const int32_t *__restrict__ rho,
                                                      const int32_t *__restrict__ bstart,
                                                      const double *__restrict__ bd,
                                                      const int32_t *__restrict__ bi,
                                                      uint8_t *__restrict__ selflag,
                                                      const DevScalars *__restrict__ sc) {
    if (sc->err) return;
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= H || rho[j] != 0) return;
    const int32_t b0 = bstart[j], b1 = bstart[j + 1];
    if (b1 <= b0) return;
    double d = DBL_MAX;
    int32_t i = INT32_MAX;
    for (int32_t q = b0 + (int32_t)lane_id(); q < b1; q += kWave) {
        const double dq = bd[q];
        const int32_t iq = bi[q];
        if (dq < d || (dq == d && iq < i)) { d = dq; i = iq; }
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double dq = __shfl_xor(d, o, 64);
        const int32_t iq = __shfl_xor(i, o, 64);
        if (dq < d || (dq == d && iq < i)) { d = dq; i = iq; }
    }
    if (lane_id() == 0) selflag[i] = 2;
}

// Per tile of kOsTile indices: number of picks (flag 2) and of unpicked
// last-front members, in cnt[0 .. nb) and cnt[nbp .. nbp + nb).
__global__ __launch_bounds__(256) void k_oneshot_count(int64_t N, const int32_t *__restrict__ rank,
                                                       const uint8_t *__restrict__ selflag,
                                                       uint32_t *__restrict__ cnt, int64_t nbp,
                                                       const DevScalars *__restrict__ sc) {
    __shared__ uint32_t red[2][4];
    if (sc->err) return;
    const int32_t l = sc->last_front;
    const int64_t base = (int64_t)blockIdx.x * kOsTile;
    uint32_t cp = 0, cq = 0;
#pragma unroll
    for (int it = 0; it < kOsTile / 256; ++it) {
        const int64_t p = base + it * 256 + threadIdx.x;
        if (p < N) {
            const uint8_t f = selflag[p];
            cp += f == 2 ? 1u : 0u;
            cq += (f != 2 && rank[p] == l) ? 1u : 0u;
        }
    }
    cp = wave_sum(cp);
    cq = wave_sum(cq);
    if (lane_id() == 0) {
        red[0][threadIdx.x / kWave] = cp;
        red[1][threadIdx.x / kWave] = cq;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        cnt[blockIdx.x] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        cnt[nbp + blockIdx.x] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// Final flags: a pick stays when R >= |E| or fewer than R picks precede it; an
// unpicked last-front member is added when fewer than R - |E| of them precede
// it.  off holds the exclusive tile prefixes of both counts (as cnt above);
// totals[0] = |E|.
__global__ __launch_bounds__(256) void k_oneshot_apply(int64_t N, const int32_t *__restrict__ rank,
                                                       uint8_t *__restrict__ selflag,
                                                       const uint32_t *__restrict__ off, int64_t nbp,
                                                       const uint32_t *__restrict__ totals,
                                                       const DevScalars *__restrict__ sc) {
    __shared__ uint32_t lds[5];
    if (sc->err) return;
    const int32_t l = sc->last_front;
    const int64_t R = sc->num_from_last;
    const int64_t ne = totals[0];
    const int64_t base = (int64_t)blockIdx.x * kOsTile;
    int64_t op = off[blockIdx.x], oq = off[nbp + blockIdx.x];
    for (int it = 0; it < kOsTile / 256; ++it) {
        const int64_t p = base + it * 256 + threadIdx.x;
        uint8_t f = 0;
        bool member = false;
        if (p < N) {
            f = selflag[p];
            member = rank[p] == l;
        }
        const uint32_t isP = f == 2 ? 1u : 0u;
        const uint32_t isQ = (member && f != 2) ? 1u : 0u;
        // picks in the low 16 bits, unpicked members in the high ones (<= 256 each)
        uint32_t tot;
        const uint32_t ex = block_exclusive_scan(isP | (isQ << 16), lds, &tot);
        if (isP) selflag[p] = (R >= ne || op + (ex & 0xffffu) < R) ? 1 : 0;
        if (isQ) selflag[p] = (R > ne && oq + (ex >> 16) < R - ne) ? 1 : 0;
        op += tot & 0xffffu;
        oq += tot >> 16;
    }
}

size_t oneshot_temp_bytes(int64_t n) {
    const int64_t nb = (n + kOsTile - 1) / kOsTile;
    return (size_t)(2 * (nb + 64) + 64) * sizeof(uint32_t);
}

void run_finalize(nsga3_info *info, int64_t K, const DevScalars *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, info, K, sc);
}

int normalize_partial_blocks(int64_t N) {
    int64_t nb = (N + kNormThreads - 1) / kNormThreads;
    if (nb > kNormBlocksMax) nb = kNormBlocksMax;
    if (nb < 1) nb = 1;
    return (int)nb;
}

hipError_t run_select_stage(const SelectViews &v, hipStream_t s) {
    const int64_t N = v.N;
    const int M = v.M;
    const int nparts = normalize_partial_blocks(N);
    v.mark();
    hipLaunchKernelGGL(k_extreme_partial, dim3(nparts), dim3(kNormThreads), 0, s, v.objs, N, M,
                       v.rank, v.sc, v.p_asf, v.p_idx, v.p_nad);
    switch (M) {
#define NSGA3_CASE(m)                                                                               \
    case m:                                                                                         \
        hipLaunchKernelGGL(k_solve<m>, dim3(1), dim3(kSolveThreads), 0, s, v.objs, nparts, v.p_asf, \
                           v.p_idx, v.p_nad, v.sc);                                                 \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    const unsigned nbN = (unsigned)((N + 255) / 256);
    v.mark();
    const unsigned nbW = (unsigned)((N + 127) / 128);  // 32 points per wave, 4 waves per block
    switch (M) {
#define NSGA3_CASE(m)                                                                               \
    case m:                                                                                         \
        if (v.assoc_mode == NSGA3_ASSOC_BF16)                                                       \
            hipLaunchKernelGGL(k_associate_bf16<m>, dim3(nbW), dim3(256), 0, s, v.objs, N, v.rank,  \
                               v.rhat64, v.rhat16, v.H, v.niche, v.dist, v.dist64, v.rho,           \
                               v.bcount, v.selflag, v.sc);                                          \
        else                                                                                        \
            hipLaunchKernelGGL(k_associate<m>, dim3(nbN), dim3(kNormThreads), 0, s, v.objs, N,      \
                               v.rank, v.rhat64, v.rhat32, v.H, v.niche, v.dist, v.dist64, v.rho,   \
                               v.bcount, v.selflag, v.sc);                                          \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    v.mark();
    hipLaunchKernelGGL(k_niche_plan, dim3(1), dim3(1024), 0, s, v.H, v.rho, v.bcount, v.bstart,
                       v.bcursor, v.gstart, v.sc);
    hipLaunchKernelGGL(k_bucket_scatter, dim3(nbN), dim3(256), 0, s, N, v.H, v.rank, v.niche, v.dist64,
                       v.bcursor, v.bd, v.bi, v.sc);
    if (v.niching_mode == NSGA3_NICHING_ONESHOT) {
        hipLaunchKernelGGL(k_oneshot_pick, dim3((unsigned)((v.H + 3) / 4)), dim3(256), 0, s, v.H,
                           v.rho, v.bstart, v.bd, v.bi, v.selflag, v.sc);
        const int64_t nbo = (N + kOsTile - 1) / kOsTile;
        const int64_t nbp = nbo + 64;
        uint32_t *cnt = v.temp, *totals = v.temp + 2 * nbp;
        hipLaunchKernelGGL(k_oneshot_count, dim3((unsigned)nbo), dim3(256), 0, s, N, v.rank,
                           v.selflag, cnt, nbp, v.sc);
        scan_inplace(cnt, nbo, totals, s);
        scan_inplace(cnt + nbp, nbo, totals + 1, s);
        hipLaunchKernelGGL(k_oneshot_apply, dim3((unsigned)nbo), dim3(256), 0, s, N, v.rank,
                           v.selflag, cnt, nbp, totals, v.sc);
    } else {
        // at most ceil(|F_l| / kRankMembers) + H groups, |F_l| <= N
        const unsigned nbG = (unsigned)((N + kRankMembers - 1) / kRankMembers + v.H);
        hipLaunchKernelGGL(k_bucket_rank, dim3(nbG), dim3(kRankGroup), 0, s, v.H, v.rho, v.bstart,
                           v.gstart, v.bd, v.bi, v.selflag, v.sc);
    }
    compact_flags(v.selflag, N, v.selected, v.K, v.temp, &v.sc->n_selected, s);
    if (v.info) hipLaunchKernelGGL(k_finalize, dim3(1), dim3(64), 0, s, v.info, v.K, v.sc);
    v.mark();
    return hipGetLastError();
}

hipError_t run_refs(const float *refs, int H, int M, double *rhat64, float *rhat32,
                    uint16_t *rhat16, DevScalars *sc, hipStream_t s) {
    const int Hpad = (H + 31) / 32 * 32;
    const int KP = M <= 8 ? 8 : 16;
    hipLaunchKernelGGL(k_refs, dim3((Hpad + 255) / 256), dim3(256), 0, s, refs, H, M, rhat64,
                       rhat32, rhat16, Hpad, KP, sc);
    return hipGetLastError();
}

}  // namespace nsga3
