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

// a5: intercepts from the extreme points (one thread).  e[j] is the index of
// the extreme point of axis j, nadir[k] the largest translated value over S.
// Solves E b = 1 by Gaussian elimination with partial pivoting (largest
// |pivot|, lowest row on ties; singular when a pivot is <= 1e-10 max|E|);
// a = 1/b when every b_k is finite and positive and every 1/b_k finite, else
// the nadir; an intercept of exactly 0 becomes 1.  Returns the fallback code
// (0 hyperplane, 1 nadir, 2 unit guard).
__device__ inline int solve_intercepts(const float *objs, int M, const int32_t *e,
                                       const double *nadir, const double *z, double *a) {
    double A[16 * 16], rhs[16], b[16];
    double maxabs = 0.0;
    for (int j = 0; j < M; ++j) {
        for (int k = 0; k < M; ++k) {
            const double v = (double)objs[(int64_t)e[j] * M + k] - z[k];
            A[j * M + k] = v;
            const double av = fabs(v);
            if (av > maxabs) maxabs = av;
        }
        rhs[j] = 1.0;
    }
    bool ok = maxabs > 0.0;
    for (int c = 0; c < M && ok; ++c) {
        int p = c;
        double pv = fabs(A[c * M + c]);
        for (int r = c + 1; r < M; ++r) {
            const double v = fabs(A[r * M + c]);
            if (v > pv) { pv = v; p = r; }
        }
        if (!(pv > 1e-10 * maxabs)) { ok = false; break; }
        if (p != c) {
            for (int k = 0; k < M; ++k) {
                const double t = A[c * M + k];
                A[c * M + k] = A[p * M + k];
                A[p * M + k] = t;
            }
            const double t = rhs[c]; rhs[c] = rhs[p]; rhs[p] = t;
        }
        for (int r = c + 1; r < M; ++r) {
            const double f = A[r * M + c] / A[c * M + c];
            for (int k = c + 1; k < M; ++k) A[r * M + k] = A[r * M + k] - f * A[c * M + k];
            A[r * M + c] = 0.0;
            rhs[r] = rhs[r] - f * rhs[c];
        }
    }
    if (ok) {
        for (int c = M - 1; c >= 0; --c) {
            double s = rhs[c];
            for (int k = c + 1; k < M; ++k) s = s - A[c * M + k] * b[k];
            b[c] = s / A[c * M + c];
        }
        for (int k = 0; k < M && ok; ++k) {
            if (!(__builtin_isfinite(b[k]) && b[k] > 0.0)) { ok = false; break; }
            const double ak = 1.0 / b[k];
            if (!__builtin_isfinite(ak)) { ok = false; break; }
            a[k] = ak;
        }
    }
    int fb = 0;
    if (!ok) {
        fb = 1;
        for (int k = 0; k < M; ++k) a[k] = nadir[k];
    }
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
template <int M>
__device__ __forceinline__ void associate_point(const double (&fp)[M], const float (&y)[M], float l1,
                                                const float *R, const double *rhat64, int H,
                                                int32_t &best, double &d1, double &d2) {
    float smax = -FLT_MAX;
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < M; ++k) s = __fmaf_rn(y[k], R[j * M + k], s);
        smax = s > smax ? s : smax;
    }
    const float thr = smax - fp32_band<M>(l1);
    d1 = DBL_MAX;
    d2 = DBL_MAX;
    best = 0;
    for (int j = 0; j < H; ++j) {
        float s = 0.0f;
#pragma unroll
        for (int k = 0; k < M; ++k) s = __fmaf_rn(y[k], R[j * M + k], s);
        if (s < thr) continue;
        const double d = line_distance<M>(fp, rhat64 + (int64_t)j * M);
        if (d < d1) { d2 = d1; d1 = d; best = j; }
        else if (d < d2) { d2 = d; }
    }
}

// Near-tie rule: the two smallest distances differ by less than 1e-6 relative.
__device__ __forceinline__ bool near_tie(double d1, double d2) {
    return d2 != DBL_MAX && (d2 - d1) < 1e-6 * fmax(d2, 1e-300);
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
