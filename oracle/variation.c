/*
 * CPU oracle for the tensorized variation operators and the gather around the
 * selection -- TEST INFRASTRUCTURE ONLY (plain float64 C; shares no code with
 * the GPU path).
 *
 * Paper: "Bridging Evolutionary Multiobjective Optimization and GPU
 * Acceleration via Tensorization" (Liang et al., IEEE TEVC 2025),
 * Supplementary Sec. S.I: simulated binary crossover (Eq. (S.6)-(S.7)) and
 * polynomial mutation (Eq. (S.8)-(S.11)); Eq. (13) for the gather of the
 * selected rows.
 *
 * SBX: the n x d population X is split into X1 = rows [0, h) and X2 = rows
 * [h, 2h), h = floor(n / 2); with a uniform draw m per (row, variable),
 *   B = (2m)^(1/(eta_c+1))          if m <= 1/2
 *     = (1/(2 - 2m))^(1/(eta_c+1))  otherwise,
 *   child 1 = ((1 + B) x1 + (1 - B) x2) / 2, child 2 = ((1 - B) x1 + (1 + B) x2) / 2
 * (children of row r at rows r and h + r).  Polynomial mutation of every
 * child variable x with a draw m, eta = eta_m + 1, D = u - l:
 *   d1 = (x - l) / D, d2 = (u - x) / D,
 *   step = (2m + (1 - 2m)(1 - d1)^eta)^(1/eta) - 1        if m <= 1/2
 *        = 1 - (2 - 2m + (2m - 1)(1 - d2)^eta)^(1/eta)    otherwise,
 *   x' = x + step D.
 * Readings (listed in the design notes):
 *   - the printed first step lacks the "- 1" of the polynomial mutation (as
 *     printed it could never decrease a variable): it is restored;
 *   - children are clipped to [l, u] before the mutation (the normalised
 *     distances d1, d2 must lie in [0, 1]);
 *   - every variable is mutated (the printed form has no mutation mask);
 *   - the draws are inputs, in [0, 1); odd n leaves the last row unused.
 * Return codes: 0 ok, -1 invalid argument, -2 non-finite input or l >= u.
 */
#include <math.h>
#include <stdint.h>

int oracle_sbx_pm(const float *X, int64_t n, int d, const float *lower, const float *upper,
                  double eta_c, double eta_m, const float *r_sbx, const float *r_pm, double *out)
{
    if (!X || !lower || !upper || !r_sbx || !r_pm || !out || n < 2 || d < 1 || !(eta_c >= 0.0) ||
        !(eta_m >= 0.0) || !isfinite(eta_c) || !isfinite(eta_m))
        return -1;
    const int64_t h = n / 2;
    for (int j = 0; j < d; ++j)
        if (!isfinite(lower[j]) || !isfinite(upper[j]) || !(lower[j] < upper[j])) return -2;
    for (int64_t q = 0; q < 2 * h * d; ++q)
        if (!isfinite(X[q]) || !isfinite(r_pm[q])) return -2;
    for (int64_t q = 0; q < h * d; ++q)
        if (!isfinite(r_sbx[q])) return -2;
    const double ec = 1.0 / (eta_c + 1.0);
    const double eta = eta_m + 1.0;
    #pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < h; ++r) {
        for (int j = 0; j < d; ++j) {
            const double x1 = (double)X[r * d + j], x2 = (double)X[(h + r) * d + j];
            const double m = (double)r_sbx[r * d + j];
            const double B = m <= 0.5 ? pow(2.0 * m, ec) : pow(1.0 / (2.0 - 2.0 * m), ec);
            double c[2];
            c[0] = ((1.0 + B) * x1 + (1.0 - B) * x2) / 2.0;
            c[1] = ((1.0 - B) * x1 + (1.0 + B) * x2) / 2.0;
            const double lo = (double)lower[j], hi = (double)upper[j], D = hi - lo;
            for (int t = 0; t < 2; ++t) {
                const int64_t row = t == 0 ? r : h + r;
                double x = c[t] < lo ? lo : (c[t] > hi ? hi : c[t]);
                const double mm = (double)r_pm[row * d + j];
                double step;
                if (mm <= 0.5) {
                    const double d1 = (x - lo) / D;
                    step = pow(2.0 * mm + (1.0 - 2.0 * mm) * pow(1.0 - d1, eta), 1.0 / eta) - 1.0;
                } else {
                    const double d2 = (hi - x) / D;
                    step = 1.0 - pow(2.0 - 2.0 * mm + (2.0 * mm - 1.0) * pow(1.0 - d2, eta), 1.0 / eta);
                }
                out[row * d + j] = x + step * D;
            }
        }
    }
    return 0;
}

/* Eq. (13): out row q = X row idx[q]. */
int oracle_gather_rows(const float *X, int64_t N, int d, const int32_t *idx, int64_t K, float *out)
{
    if (!X || !idx || !out || N < 1 || d < 1 || K < 0) return -1;
    for (int64_t q = 0; q < K; ++q)
        if (idx[q] < 0 || idx[q] >= N) return -1;
    for (int64_t q = 0; q < K; ++q)
        for (int j = 0; j < d; ++j) out[q * d + j] = X[(int64_t)idx[q] * d + j];
    return 0;
}
