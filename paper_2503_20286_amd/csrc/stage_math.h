// Per-point and per-instance arithmetic of the selection stages (internal),
// shared by the single-selection kernels and the batched engine so that both
// produce bit-identical results.
#pragma once

#include <float.h>

#include "common.h"

namespace nsga3 {

// a4: achievement scalarising function of one translated point g (Alg. S.5,
// weights 1 on axis j and 1e-6 elsewhere, applied as x 1e6) for every axis j,
// folded into running minima (lowest index on ties) and the nadir maxima.
template <int MM>
__device__ __forceinline__ void asf_fold(const double (&g)[MM], int M, int32_t i, double (&best)[MM],
                                         int32_t (&bidx)[MM], double (&nad)[MM]) {
#pragma unroll
    for (int k = 0; k < MM; ++k)
        if (k < M && g[k] > nad[k]) nad[k] = g[k];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
        if (j < M) {
            double asf = -DBL_MAX;
#pragma unroll
            for (int k = 0; k < MM; ++k) {
                if (k < M) {
                    const double v = (k == j) ? g[k] : g[k] * 1e6;
                    if (v > asf) asf = v;
                }
            }
            if (asf < best[j]) { best[j] = asf; bidx[j] = i; }
        }
    }
}

// a5: intercepts from the extreme points, by one whole wave (lane r holds
// row r of E; lanes >= M only take part in the shuffles).  e[j] is the index
// of the extreme point of axis j, nadir[k] the largest translated value over
// S, z the ideal point.  Solves E b = 1 by Gaussian elimination with partial
// pivoting (largest |pivot|, lowest row on ties; singular when a pivot is
// <= 1e-10 max|E|); a = 1/b when every b_k is finite and positive and every
// 1/b_k finite, else the nadir; an intercept of exactly 0 becomes 1.  Every
// lane returns the same a and fallback code (0 hyperplane, 1 nadir, 2 unit
// guard).  Each entry goes through the same operations, in the same order, as
// in the one-row-at-a-time textbook elimination.
template <int M>
__device__ __forceinline__ int solve_intercepts_wave(const float *objs, const int32_t *e,
                                                     const double *nadir, const double (&z)[M],
                                                     double (&a)[M]) {
    const int lane = (int)lane_id();
    const bool own = lane < M;
    const int64_t er = e[own ? lane : 0];
    double row[M];
    double rhs = 1.0;
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        row[k] = (double)objs[er * M + k] - z[k];
        const double av = fabs(row[k]);
        mx = av > mx ? av : mx;
    }
    double maxabs = own ? mx : 0.0;
    for (int o = 32; o > 0; o >>= 1) {
        const double t = __shfl_xor(maxabs, o, 64);
        maxabs = t > maxabs ? t : maxabs;
    }
    bool ok = maxabs > 0.0;
#pragma unroll
    for (int c = 0; c < M; ++c) {
        double pv = (own && lane >= c) ? fabs(row[c]) : -1.0;
        int p = lane;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(pv, o, 64);
            const int op = __shfl_xor(p, o, 64);
            if (ov > pv || (ov == pv && op < p)) { pv = ov; p = op; }
        }
        ok = ok && pv > 1e-10 * maxabs;
        // rows c and p trade places
        const int src = lane == c ? p : (lane == p ? c : lane);
#pragma unroll
        for (int k = c; k < M; ++k) row[k] = __shfl(row[k], src, 64);
        rhs = __shfl(rhs, src, 64);
        double prow[M];
#pragma unroll
        for (int k = c; k < M; ++k) prow[k] = __shfl(row[k], c, 64);
        const double prhs = __shfl(rhs, c, 64);
        if (own && lane > c) {
            const double f = row[c] / prow[c];
#pragma unroll
            for (int k = c + 1; k < M; ++k) row[k] = row[k] - f * prow[k];
            row[c] = 0.0;
            rhs = rhs - f * prhs;
        }
    }
    if (ok) {
        double b[M];
#pragma unroll
        for (int c = M - 1; c >= 0; --c) {
            double s = __shfl(rhs, c, 64);
#pragma unroll
            for (int k = c + 1; k < M; ++k) s = s - __shfl(row[k], c, 64) * b[k];
            b[c] = s / __shfl(row[c], c, 64);
        }
#pragma unroll
        for (int k = 0; k < M; ++k) {
            if (!(ok && __builtin_isfinite(b[k]) && b[k] > 0.0)) { ok = false; continue; }
            const double ak = 1.0 / b[k];
            if (!__builtin_isfinite(ak)) ok = false;
            a[k] = ak;
        }
    }
    int fb = 0;
    if (!ok) {
        fb = 1;
#pragma unroll
        for (int k = 0; k < M; ++k) a[k] = nadir[k];
    }
#pragma unroll
    for (int k = 0; k < M; ++k)
        if (a[k] == 0.0) { a[k] = 1.0; fb = 2; }
    return fb;
}

// a6: normalised point f' = (f - z) / a and its screening vector y = f' / max f'
// (the scale of y does not move the argmax of y . rhat).  Returns ||y||_1.
template <int M>
__device__ __forceinline__ float normalise_point(const float *f, const double *z, const double *a,
                                                 double (&fp)[M], float (&y)[M]) {
    double mx = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        fp[k] = ((double)f[k] - z[k]) / a[k];
        mx = fp[k] > mx ? fp[k] : mx;
    }
    float l1 = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        y[k] = mx > 0.0 ? (float)(fp[k] / mx) : 0.0f;
        l1 += y[k];
    }
    return l1;
}

// Float64 residual distance of f' to the line of unit reference rd (Eq. (10)
// in its residual form ||f' - (f'.r) r||).
template <int M>
__device__ __forceinline__ double line_distance(const double (&fp)[M], const double *rd) {
    double s64 = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) s64 = s64 + fp[k] * rd[k];
    double q = 0.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const double e = fp[k] - s64 * rd[k];
        q = q + e * e;
    }
    return sqrt(q);
}

// Float32 screening band: |s32 - s| <= (M + 3) u ||y||_2 <= (M + 3) u ||y||_1
// with u = 2^-24; a 4x margin keeps every reference within float64 reach of
// the best one.
template <int M>
__device__ __forceinline__ float fp32_band(float l1) {
    return 4.0f * (float)(M + 4) * 5.9604645e-8f * l1 + 1e-30f;
}

// a6 for one point: screen every reference with s = y . rhat in float32 (R is
// the H x M float32 unit references), re-score the survivors in float64.
// best = lowest index among the smallest distances; d1 <= d2 the two smallest.
// References go four at a time (independent chains; each s is summed in the
// same order as a one-at-a-time loop, and survivors are visited in ascending
// index order, so results do not depend on the grouping).
template <int M>
__device__ __forceinline__ float screen_dot(const float (&y)[M], const float *__restrict__ r) {
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < M; ++k) s = __fmaf_rn(y[k], r[k], s);
    return s;
}

template <int M>
__device__ __forceinline__ void associate_point(const double (&fp)[M], const float (&y)[M], float l1,
                                                const float *__restrict__ R,
                                                const double *__restrict__ rhat64, int H,
                                                int32_t &best, double &d1, double &d2) {
    float smax = -FLT_MAX;
    int j = 0;
    for (; j + 4 <= H; j += 4) {
        const float s0 = screen_dot<M>(y, R + (j + 0) * M), s1 = screen_dot<M>(y, R + (j + 1) * M);
        const float s2 = screen_dot<M>(y, R + (j + 2) * M), s3 = screen_dot<M>(y, R + (j + 3) * M);
        smax = fmaxf(smax, fmaxf(fmaxf(s0, s1), fmaxf(s2, s3)));
    }
    for (; j < H; ++j) smax = fmaxf(smax, screen_dot<M>(y, R + j * M));
    const float thr = smax - fp32_band<M>(l1);
    d1 = DBL_MAX;
    d2 = DBL_MAX;
    best = 0;
    auto consider = [&](int jj, float s) {
        if (s < thr) return;
        const double d = line_distance<M>(fp, rhat64 + (int64_t)jj * M);
        if (d < d1) { d2 = d1; d1 = d; best = jj; }
        else if (d < d2) { d2 = d; }
    };
    j = 0;
    for (; j + 4 <= H; j += 4) {
        const float s0 = screen_dot<M>(y, R + (j + 0) * M), s1 = screen_dot<M>(y, R + (j + 1) * M);
        const float s2 = screen_dot<M>(y, R + (j + 2) * M), s3 = screen_dot<M>(y, R + (j + 3) * M);
        consider(j, s0);
        consider(j + 1, s1);
        consider(j + 2, s2);
        consider(j + 3, s3);
    }
    for (; j < H; ++j) consider(j, screen_dot<M>(y, R + j * M));
}

// Near-tie rule: the two smallest distances differ by less than 1e-6 relative.
__device__ __forceinline__ bool near_tie(double d1, double d2) {
    return d2 != DBL_MAX && (d2 - d1) < 1e-6 * fmax(d2, 1e-300);
}

// a7 niche counts of one work-group.  cls = 0 counts reference `best` into
// rho, cls = 1 into bcount, cls < 0 counts nothing.  For H <= kLdsNicheRefs the
// work-group first tallies in LDS (hist: 2 * kLdsNicheRefs ints) and then adds
// each non-zero tally with one global atomic, so a popular reference takes one
// atomic per work-group instead of one per point.  Every thread of the
// work-group calls it; it ends with a barrier.
constexpr int kLdsNicheRefs = 2048;

__device__ __forceinline__ void niche_count_block(int H, int cls, int32_t best, int32_t *rho,
                                                  int32_t *bcount, int32_t *hist) {
    if (H <= kLdsNicheRefs) {
        for (int q = threadIdx.x; q < 2 * H; q += blockDim.x) hist[q] = 0;
        __syncthreads();
        if (cls >= 0) atomicAdd(&hist[cls * H + best], 1);
        __syncthreads();
        for (int q = threadIdx.x; q < 2 * H; q += blockDim.x) {
            const int32_t v = hist[q];
            if (v) atomicAdd(q < H ? &rho[q] : &bcount[q - H], v);
        }
        __syncthreads();
    } else if (cls >= 0) {
        atomicAdd(cls ? &bcount[best] : &rho[best], 1);
    }
}

// a8 bucket slot of one work-group's last-front members (member: this thread
// holds one, in bucket b).  With H <= kLdsNicheRefs each bucket's cursor takes
// one atomic per work-group (cnt: kLdsNicheRefs ints of LDS).  Every thread of
// the work-group calls it; it ends with a barrier.  Slots inside a bucket are
// in no particular order.
__device__ __forceinline__ int32_t bucket_slot_block(int H, bool member, int32_t b,
                                                     int32_t *bcursor, int32_t *cnt) {
    if (H > kLdsNicheRefs) return member ? atomicAdd(&bcursor[b], 1) : -1;
    for (int q = threadIdx.x; q < H; q += blockDim.x) cnt[q] = 0;
    __syncthreads();
    const int32_t local = member ? atomicAdd(&cnt[b], 1) : 0;
    __syncthreads();
    for (int q = threadIdx.x; q < H; q += blockDim.x) {
        const int32_t v = cnt[q];
        if (v) cnt[q] = atomicAdd(&bcursor[q], v);
    }
    __syncthreads();
    const int32_t slot = member ? cnt[b] + local : -1;
    __syncthreads();
    return slot;
}

// Unit reference j (float64, float32); false when the row is invalid
// (non-finite, negative entry, zero norm).
__device__ __forceinline__ bool unit_reference(const float *refs, int j, int M, double *r64,
                                               float *r32) {
    double nn = 0.0;
    bool bad = false;
    for (int k = 0; k < M; ++k) {
        const float f = refs[(int64_t)j * M + k];
        bad |= !__builtin_isfinite(f) || f < 0.0f;
        const double v = (double)f;
        nn = nn + v * v;
    }
    const double n = sqrt(nn);
    bad |= !(n > 0.0) || !__builtin_isfinite(n);
    if (bad) return false;
    for (int k = 0; k < M; ++k) {
        const double r = (double)refs[(int64_t)j * M + k] / n;
        r64[(int64_t)j * M + k] = r;
        r32[(int64_t)j * M + k] = (float)r;
    }
    return true;
}

}  // namespace nsga3
