/*
 * CPU oracle for the TensorRVEA environmental selection -- TEST
 * INFRASTRUCTURE ONLY (plain float64 C; shares no code with the GPU path).
 *
 * Paper: "Bridging Evolutionary Multiobjective Optimization and GPU
 * Acceleration via Tensorization" (Liang et al., IEEE TEVC 2025),
 * Supplementary Sec. S.V, Alg. S.12 (environmental selection of TensorRVEA).
 *
 * The selection keeps one elite per reference vector:
 *   z = min_i F_i (per objective, over the whole population),  F' = F - z;
 *   theta_ij = angle between F'_i and reference V_j;
 *   a_i = the reference with the smallest angle (the partition of point i);
 *   gamma_j = the smallest angle between V_j and any other reference;
 *   APD_i = (1 + M (t / t_max)^alpha theta_{i,a_i} / gamma_{a_i}) ||F'_i||;
 *   elite_j = the point of partition j with the smallest APD, or -1 when the
 *             partition is empty.
 * Readings of points the algorithm leaves open (listed in the design notes):
 *   - the smallest angle is the largest dot product F'_i . V_j / ||V_j||
 *     (arccos is decreasing); the partition is decided on that dot product,
 *     lowest j on ties;
 *   - Gamma is read as the smallest angle to another reference (the printed
 *     argmin over the angle matrix would return an index and include each
 *     vector's zero angle to itself); two equal reference directions make it
 *     0 and are rejected like an invalid reference row;
 *   - a point equal to the ideal point (F' = 0) has no direction: it joins
 *     partition 0 with angle 0 and APD 0;
 *   - argmin ties between equal APDs go to the lowest point index;
 *   - the penalty factor M (t / t_max)^alpha is computed once in float64.
 * Return codes: 0 ok, -1 invalid argument, -2 non-finite input or invalid
 * reference row (negative entry, zero norm, or a duplicate direction).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Unit reference vectors (float64), or -2 for a bad row. */
static int unit_refs(const float *refs, int H, int M, double *rhat)
{
    for (int j = 0; j < H; ++j) {
        double nn = 0.0;
        for (int k = 0; k < M; ++k) {
            const double v = (double)refs[j * M + k];
            if (!isfinite(v) || v < 0.0) return -2;
            nn = nn + v * v;
        }
        const double n = sqrt(nn);
        if (!(n > 0.0)) return -2;
        for (int k = 0; k < M; ++k) rhat[j * M + k] = (double)refs[j * M + k] / n;
    }
    return 0;
}

/* gamma_j = min over k != j of the angle between V_j and V_k (Alg. S.12,
 * the Gamma line).  Needs H >= 2. */
int oracle_rvea_gamma(const float *refs, int H, int M, double *gamma)
{
    if (!refs || !gamma || H < 2 || M < 1) return -1;
    double *rhat = (double *)malloc(sizeof(double) * (size_t)H * (size_t)M);
    if (!rhat) return -1;
    int rc = unit_refs(refs, H, M, rhat);
    for (int j = 0; j < H && rc == 0; ++j) {
        double best = -2.0;   /* largest cosine to another reference */
        for (int q = 0; q < H; ++q) {
            if (q == j) continue;
            double c = 0.0;
            for (int k = 0; k < M; ++k) c = c + rhat[j * M + k] * rhat[q * M + k];
            if (c > best) best = c;
        }
        gamma[j] = acos(best > 1.0 ? 1.0 : best);
        if (!(gamma[j] > 0.0)) rc = -2;    /* a duplicate direction */
    }
    free(rhat);
    return rc;
}

/* The whole selection.  elite[H] required; assign[N], apd[N], theta[N] and
 * gap[H] optional.  gap_j = (second smallest - smallest APD) / second smallest
 * in partition j (1 when it has one member, -1 when empty). */
int oracle_rvea_select(const float *objs, int64_t N, int M, const float *refs, int H,
                       int64_t t, int64_t t_max, double alpha, int32_t *elite,
                       int32_t *assign, double *apd, double *theta, double *gap)
{
    if (!objs || !refs || !elite || N < 1 || M < 1 || M > 64 || H < 2 || t < 0 || t_max < 1 ||
        !(alpha >= 0.0) || !isfinite(alpha))
        return -1;
    for (int64_t q = 0; q < N * M; ++q)
        if (!isfinite(objs[q])) return -2;
    const size_t n = (size_t)N;
    double *rhat = (double *)malloc(sizeof(double) * (size_t)H * (size_t)M);
    double *gamma = (double *)malloc(sizeof(double) * (size_t)H);
    int32_t *a = (int32_t *)malloc(sizeof(int32_t) * n);
    double *ap = (double *)malloc(sizeof(double) * n);
    double *th = (double *)malloc(sizeof(double) * n);
    int rc = 0;
    if (!rhat || !gamma || !a || !ap || !th) { rc = -1; goto done; }
    rc = unit_refs(refs, H, M, rhat);
    if (rc) goto done;
    rc = oracle_rvea_gamma(refs, H, M, gamma);
    if (rc) goto done;
    double z[64];
    for (int k = 0; k < M; ++k) z[k] = INFINITY;
    for (size_t i = 0; i < n; ++i)
        for (int k = 0; k < M; ++k) {
            const double v = (double)objs[i * M + k];
            if (v < z[k]) z[k] = v;
        }
    const double penalty = (double)M * pow((double)t / (double)t_max, alpha);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        double f[64];
        double nn = 0.0;
        for (int k = 0; k < M; ++k) {
            f[k] = (double)objs[i * M + k] - z[k];
            nn = nn + f[k] * f[k];
        }
        const double norm = sqrt(nn);
        if (!(norm > 0.0)) {            /* the ideal point itself */
            a[i] = 0;
            th[i] = 0.0;
            ap[i] = 0.0;
            continue;
        }
        double best = -INFINITY;        /* largest F' . V_j / ||V_j|| */
        int32_t bj = 0;
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k) s = s + f[k] * rhat[j * M + k];
            if (s > best) { best = s; bj = j; }
        }
        double c = best / norm;
        if (c > 1.0) c = 1.0;
        const double ang = acos(c);
        a[i] = bj;
        th[i] = ang;
        ap[i] = (1.0 + penalty * ang / gamma[bj]) * norm;
    }
    for (int j = 0; j < H; ++j) elite[j] = -1;
    for (size_t i = 0; i < n; ++i) {
        const int32_t j = a[i];
        if (elite[j] < 0 || ap[i] < ap[elite[j]]) elite[j] = (int32_t)i;
    }
    if (gap) {
        for (int j = 0; j < H; ++j) gap[j] = elite[j] < 0 ? -1.0 : 1.0;
        for (size_t i = 0; i < n; ++i) {
            const int32_t j = a[i];
            if ((int32_t)i == elite[j]) continue;
            const double d = (ap[i] - ap[elite[j]]) / (ap[i] > 0.0 ? ap[i] : 1.0);
            if (d < gap[j]) gap[j] = d;
        }
    }
    for (size_t i = 0; i < n; ++i) {
        if (assign) assign[i] = a[i];
        if (apd) apd[i] = ap[i];
        if (theta) theta[i] = th[i];
    }
done:
    free(rhat); free(gamma); free(a); free(ap); free(th);
    return rc;
}
