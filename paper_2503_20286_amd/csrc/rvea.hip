// Environmental selection of TensorRVEA (Supplementary Sec. S.V, Alg. S.12):
// one elite per reference vector by the angle-penalized distance
//   APD_i = (1 + M (t / t_max)^alpha theta_i / gamma_{a_i}) ||F'_i||,
// F' = F - z (z the per-objective minimum), a_i the reference with the
// smallest angle theta_i to F'_i, gamma_j the smallest angle between V_j and
// another reference, elite_j = argmin APD over partition j (lowest index on
// ties; -1 for an empty partition).
//
//  k_rv_init    clears the per-call state
//  k_rv_refs    unit references (float64 for the scoring, float32 for the screen)
//  k_rv_gamma   one wave per reference: the largest cosine to another one
//  k_rv_ideal   per-objective minimum by order keys (block partials + atomics)
//  k_rv_assign  per point: the reference with the largest F'.V_j/||V_j||, found
//               by a float32 screen over every reference and a float64 re-score
//               of those within the screen's error band (the float64 sums run in
//               the same order for every candidate, so the winner and its angle
//               are those of a float64 scan); then theta = acos, the APD, and a
//               per-work-group minimum APD per reference (LDS), one atomic each
//  k_rv_elite   the lowest index whose APD equals its partition's minimum
//  k_rv_final   elites and the call's status
#include <float.h>

#include "kernels.h"
#include "prims.h"

namespace nsga3 {

constexpr int kRvThreads = 256;
constexpr int kRvLdsRefs = 2048;      // per-work-group APD minima kept in LDS up to this H

struct RvState {
    uint32_t err;
    uint32_t zkey[16];
};

__global__ void k_rv_init(int H, RvState *st, unsigned long long *best, int32_t *idx) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t == 0) st->err = 0;
    if (t < 16) st->zkey[t] = 0xffffffffu;
    for (int j = t; j < H; j += gridDim.x * blockDim.x) {
        best[j] = ~0ull;
        idx[j] = INT32_MAX;
    }
}

__global__ void k_rv_refs(const float *__restrict__ refs, int H, int M, double *__restrict__ rhat64,
                          float *__restrict__ rhat32, RvState *st) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= H) return;
    double nn = 0.0;
    bool ok = true;
    for (int k = 0; k < M; ++k) {
        const double v = (double)refs[j * M + k];
        ok = ok && isfinite(v) && v >= 0.0;
        nn = nn + v * v;
    }
    const double n = sqrt(nn);
    if (!ok || !(n > 0.0)) {
        atomicOr(&st->err, kErrBadRef);
        return;
    }
    for (int k = 0; k < M; ++k) {
        const double u = (double)refs[j * M + k] / n;
        rhat64[j * M + k] = u;
        rhat32[j * M + k] = (float)u;
    }
}

// gamma_j = acos(max_{q != j} V_j . V_q) in float64 (unit vectors); a
// duplicate direction (gamma 0) is an invalid reference set.
__global__ void k_rv_gamma(int H, int M, const double *__restrict__ rhat64, double *__restrict__ gamma,
                           RvState *st) {
    const int j = blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave;
    if (j >= H || st->err) return;
    double best = -2.0;
    for (int q = (int)lane_id(); q < H; q += kWave) {
        if (q == j) continue;
        double c = 0.0;
        for (int k = 0; k < M; ++k) c = c + rhat64[j * M + k] * rhat64[q * M + k];
        best = c > best ? c : best;
    }
    best = wave_max(best);
    if (lane_id() == 0) {
        const double g = acos(best > 1.0 ? 1.0 : best);
        gamma[j] = g;
        if (!(g > 0.0)) atomicOr(&st->err, kErrBadRef);
    }
}

template <int M>
__global__ __launch_bounds__(kRvThreads) void k_rv_ideal(const float *__restrict__ objs, int64_t N,
                                                          RvState *st) {
    __shared__ uint32_t red[M][kRvThreads / kWave];
    uint32_t mk[M];
    bool fin = true;
#pragma unroll
    for (int k = 0; k < M; ++k) mk[k] = 0xffffffffu;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
         i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int k = 0; k < M; ++k) {
            const float v = objs[i * M + k];
            fin = fin && isfinite(v);
            const uint32_t key = order_key(v);
            mk[k] = key < mk[k] ? key : mk[k];
        }
    }
    if (!fin) atomicOr(&st->err, kErrNonfiniteObj);
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const uint32_t w = wave_min(mk[k]);
        if (lane_id() == 0) red[k][threadIdx.x / kWave] = w;
    }
    __syncthreads();
    if (threadIdx.x < M) {
        uint32_t m = 0xffffffffu;
        for (int q = 0; q < kRvThreads / kWave; ++q) m = red[threadIdx.x][q] < m ? red[threadIdx.x][q] : m;
        atomicMin(&st->zkey[threadIdx.x], m);
    }
}

template <int M>
__global__ __launch_bounds__(kRvThreads) void k_rv_assign(
    const float *__restrict__ objs, int64_t N, int H, const double *__restrict__ rhat64,
    const float *__restrict__ rhat32, const double *__restrict__ gamma, double penalty,
    int32_t *__restrict__ assign, double *__restrict__ apd, unsigned long long *__restrict__ best,
    const RvState *__restrict__ st) {
    __shared__ unsigned long long lbest[kRvLdsRefs];
    if (st->err) return;
    const bool use_lds = H <= kRvLdsRefs;
    if (use_lds) {
        for (int j = threadIdx.x; j < H; j += blockDim.x) lbest[j] = ~0ull;
        __syncthreads();
    }
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        double f[M];
        double nn = 0.0, fmax = 0.0;
#pragma unroll
        for (int k = 0; k < M; ++k) {
            f[k] = (double)objs[i * M + k] - (double)key_to_float(st->zkey[k]);
            nn = nn + f[k] * f[k];
            fmax = f[k] > fmax ? f[k] : fmax;
        }
        const double norm = sqrt(nn);
        int32_t bj = 0;
        double a = 0.0;
        if (norm > 0.0) {
            // screen: y = F' / max_k F'_k in float32, s32_j = y . rhat32_j
            float y[M];
            float y1 = 0.0f;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                y[k] = (float)(f[k] / fmax);
                y1 += y[k];
            }
            float smax = -FLT_MAX;
            for (int j = 0; j < H; ++j) {
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k) s = fmaf(y[k], rhat32[j * M + k], s);
                smax = s > smax ? s : smax;
            }
            // every reference within the band of the screened maximum is
            // re-scored in float64, in index order (the first of equal scores wins)
            const float band = 4.0f * (float)(M + 4) * 5.9604645e-8f * y1;
            double sbest = -DBL_MAX;
            for (int j = 0; j < H; ++j) {
                float s = 0.0f;
#pragma unroll
                for (int k = 0; k < M; ++k) s = fmaf(y[k], rhat32[j * M + k], s);
                if (s >= smax - band) {
                    double d = 0.0;
#pragma unroll
                    for (int k = 0; k < M; ++k) d = d + f[k] * rhat64[j * M + k];
                    if (d > sbest) {
                        sbest = d;
                        bj = j;
                    }
                }
            }
            double c = sbest / norm;
            c = c > 1.0 ? 1.0 : c;
            const double theta = acos(c);
            a = (1.0 + penalty * theta / gamma[bj]) * norm;
        }
        assign[i] = bj;
        apd[i] = a;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(a);  // a >= 0
        if (use_lds)
            __hip_atomic_fetch_min(&lbest[bj], bits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        else
            atomicMin(&best[bj], bits);
    }
    if (use_lds) {
        __syncthreads();
        for (int j = threadIdx.x; j < H; j += blockDim.x)
            if (lbest[j] != ~0ull) atomicMin(&best[j], lbest[j]);
    }
}

__global__ void k_rv_elite(int64_t N, const int32_t *__restrict__ assign, const double *__restrict__ apd,
                           const unsigned long long *__restrict__ best, int32_t *__restrict__ idx,
                           const RvState *__restrict__ st) {
    if (st->err) return;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const int32_t j = assign[i];
    if ((unsigned long long)__double_as_longlong(apd[i]) == best[j]) atomicMin(&idx[j], (int32_t)i);
}

__global__ void k_rv_final(int H, const int32_t *__restrict__ idx, int32_t *__restrict__ elite,
                           nsga3_info *info, const RvState *__restrict__ st) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t e = st->err;
    if (j < H && !e) elite[j] = idx[j] == INT32_MAX ? -1 : idx[j];
    if (j == 0 && info) {
        nsga3_info v = {};
        v.status = e == 0 ? NSGA3_OK : NSGA3_E_NONFINITE;
        v.reserved = (int32_t)e;
        *info = v;
    }
}

static size_t up256(size_t b) { return (b + 255) / 256 * 256; }

size_t rvea_workspace_bytes(int64_t N, int M, int H) {
    auto up = up256;
    return up(sizeof(RvState)) + up(8 * (size_t)H * M) + up(4 * (size_t)H * M) + up(8 * (size_t)H) +
           up(8 * (size_t)H) + up(4 * (size_t)H) + up(4 * (size_t)N) + up(8 * (size_t)N);
}

hipError_t run_rvea(const RveaViews &v, hipStream_t s) {
    auto up = up256;
    char *w = (char *)v.ws;
    RvState *st = (RvState *)w;
    w += up(sizeof(RvState));
    double *rhat64 = (double *)w;
    w += up(8 * (size_t)v.H * v.M);
    float *rhat32 = (float *)w;
    w += up(4 * (size_t)v.H * v.M);
    double *gamma = (double *)w;
    w += up(8 * (size_t)v.H);
    unsigned long long *best = (unsigned long long *)w;
    w += up(8 * (size_t)v.H);
    int32_t *idx = (int32_t *)w;
    w += up(4 * (size_t)v.H);
    int32_t *assign = v.assign ? v.assign : (int32_t *)w;
    w += up(4 * (size_t)v.N);
    double *apd = v.apd ? v.apd : (double *)w;
    const int H = v.H, M = v.M;
    const int64_t N = v.N;
    const unsigned gH = (unsigned)((H + 255) / 256);
    hipLaunchKernelGGL(k_rv_init, dim3(gH), dim3(256), 0, s, H, st, best, idx);
    hipLaunchKernelGGL(k_rv_refs, dim3(gH), dim3(256), 0, s, v.refs, H, M, rhat64, rhat32, st);
    hipLaunchKernelGGL(k_rv_gamma, dim3((unsigned)((H + 3) / 4)), dim3(256), 0, s, H, M, rhat64,
                       gamma, st);
    const unsigned gN = (unsigned)((N + kRvThreads - 1) / kRvThreads);
    const unsigned gI = gN < 1024u ? gN : 1024u;
    switch (M) {
#define NSGA3_CASE(m)                                                                               \
    case m:                                                                                         \
        hipLaunchKernelGGL(k_rv_ideal<m>, dim3(gI), dim3(kRvThreads), 0, s, v.objs, N, st);         \
        hipLaunchKernelGGL(k_rv_assign<m>, dim3(gN), dim3(kRvThreads), 0, s, v.objs, N, H, rhat64,  \
                           rhat32, gamma, v.penalty, assign, apd, best, st);                       \
        break;
        NSGA3_CASE(2) NSGA3_CASE(3) NSGA3_CASE(4) NSGA3_CASE(5) NSGA3_CASE(6) NSGA3_CASE(7)
        NSGA3_CASE(8) NSGA3_CASE(9) NSGA3_CASE(10) NSGA3_CASE(11) NSGA3_CASE(12) NSGA3_CASE(13)
        NSGA3_CASE(14) NSGA3_CASE(15) NSGA3_CASE(16)
#undef NSGA3_CASE
        default: return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL(k_rv_elite, dim3(gN), dim3(256), 0, s, N, assign, apd, best, idx, st);
    hipLaunchKernelGGL(k_rv_final, dim3(gH), dim3(256), 0, s, H, idx, v.elite, v.info, st);
    return hipGetLastError();
}

}  // namespace nsga3
