/*
 * CPU oracle for the TensorHypE environmental selection -- TEST
 * INFRASTRUCTURE ONLY (plain float64 C; shares no code with the GPU path).
 *
 * Paper: "Bridging Evolutionary Multiobjective Optimization and GPU
 * Acceleration via Tensorization" (Liang et al., IEEE TEVC 2025), Sec. IV-C
 * (Eq. (19)-(23)), Supplementary Alg. S.10 (selection) and Alg. S.11
 * (hypervolume estimation by Monte Carlo sampling).
 *
 *   selection: ranks r and the last admitted front l for a population of n
 *     (as in the NSGA-III oracle); S = {r <= l}; k = |S| - n; d = the HV
 *     estimate on S (-inf elsewhere); the next population is the first n of
 *     the order (r ascending, d descending), i.e. every point of r < l and the
 *     members of F_l with the largest d.
 *   estimation over the N rows of F (n1 = N):
 *     alpha_c = (1/c) prod_{i=1}^{c-1} (k - i) / (N - i),  c = 1..k
 *     f_l = min_i F_i,  f_u = the reference point,  V = prod_j (f_u,j - f_l,j)
 *     sample i: S_i = f_l + U_i (f_u - f_l)  (U the caller's uniform draws)
 *     count_i = #{p : F_p <= S_i in every objective}
 *     HV_p = (sum over the samples i with F_p <= S_i and count_i <= k of
 *             alpha_{count_i}) V / s
 * Readings (listed in the design notes):
 *   - the estimation runs over all N rows of F as printed (the original
 *     HypE estimates over the overflowing front only);
 *   - a sample dominated by more than k points adds nothing (the alpha index
 *     past its end);
 *   - a sample point is computed in float64 and rounded to float32 once, and
 *     compared with the float32 objectives (weak dominance, H(0) = 1);
 *   - the random draws U are an input;
 *   - lexsort ties (equal rank and d) keep the lower index; the selected
 *     indices are returned in ascending order.
 * Return codes: 0 ok, -1 invalid argument, -2 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_ranks(const float *objs, int64_t N, int M, int32_t *rank, int32_t *num_fronts);
int oracle_last_front(const int32_t *rank, int64_t N, int64_t K, int32_t *l_out, int64_t *n_before,
                      int64_t *n_last);

/* alpha_c, c = 1..k, into alpha[0..k) (Alg. S.11, the lambda and alpha lines). */
int oracle_hype_alpha(int64_t k, int64_t N, double *alpha)
{
    if (k < 0 || N < 1 || k > N || (k > 0 && !alpha)) return -1;
    double prod = 1.0;                 /* prod_{i=1}^{c-1} lambda_{i+1} */
    for (int64_t c = 1; c <= k; ++c) {
        if (c > 1) prod = prod * ((double)(k - (c - 1)) / (double)(N - (c - 1)));
        alpha[c - 1] = prod / (double)c;
    }
    return 0;
}

/* Sample points (float32) of the box [f_l, f_u]. */
static void samples(const float *objs, int64_t N, int M, const float *vref, const float *U,
                    int64_t s, double *fl, float *S)
{
    for (int j = 0; j < M; ++j) fl[j] = INFINITY;
    for (int64_t p = 0; p < N; ++p)
        for (int j = 0; j < M; ++j)
            if ((double)objs[p * M + j] < fl[j]) fl[j] = (double)objs[p * M + j];
    for (int64_t i = 0; i < s; ++i)
        for (int j = 0; j < M; ++j)
            S[i * M + j] = (float)(fl[j] + (double)U[i * M + j] * ((double)vref[j] - fl[j]));
}

static int weakly_dominates(const float *f, const float *x, int M)
{
    for (int j = 0; j < M; ++j)
        if (!(f[j] <= x[j])) return 0;
    return 1;
}

/* HV estimates of every row for a given k (Alg. S.11).  hv[N] required,
 * count[s] optional. */
int oracle_hype_hv(const float *objs, int64_t N, int M, const float *vref, const float *U,
                   int64_t s, int64_t k, double *hv, int32_t *count)
{
    if (!objs || !vref || !U || !hv || N < 1 || M < 1 || M > 64 || s < 1 || k < 0 || k > N)
        return -1;
    for (int64_t q = 0; q < N * M; ++q) if (!isfinite(objs[q])) return -2;
    for (int j = 0; j < M; ++j) if (!isfinite(vref[j])) return -2;
    for (int64_t q = 0; q < s * M; ++q) if (!isfinite(U[q])) return -2;
    double *alpha = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    float *S = (float *)malloc(sizeof(float) * (size_t)s * (size_t)M);
    int32_t *cnt = (int32_t *)malloc(sizeof(int32_t) * (size_t)s);
    double *w = (double *)malloc(sizeof(double) * (size_t)s);
    if (!alpha || !S || !cnt || !w) { free(alpha); free(S); free(cnt); free(w); return -1; }
    oracle_hype_alpha(k, N, alpha);
    double fl[64];
    samples(objs, N, M, vref, U, s, fl, S);
    double V = 1.0;
    for (int j = 0; j < M; ++j) V = V * ((double)vref[j] - fl[j]);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < s; ++i) {
        int32_t c = 0;
        for (int64_t p = 0; p < N; ++p) c += weakly_dominates(objs + p * M, S + i * M, M);
        cnt[i] = c;
        w[i] = (c >= 1 && c <= k) ? alpha[c - 1] : 0.0;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < N; ++p) {
        double acc = 0.0;
        for (int64_t i = 0; i < s; ++i)
            if (weakly_dominates(objs + p * M, S + i * M, M)) acc = acc + w[i];
        hv[p] = acc * V / (double)s;
    }
    if (count) memcpy(count, cnt, sizeof(int32_t) * (size_t)s);
    free(alpha); free(S); free(cnt); free(w);
    return 0;
}

typedef struct { double d; int64_t i; } hkey_t;

static int cmp_hkey(const void *pa, const void *pb)
{
    const hkey_t *a = (const hkey_t *)pa, *b = (const hkey_t *)pb;
    if (a->d > b->d) return -1;        /* larger estimate first */
    if (a->d < b->d) return 1;
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

/* The whole selection (Alg. S.10).  selected[n] (ascending) required; d[N]
 * (the HV estimate on S, -inf elsewhere), rank[N] and info4 = [l, num_fronts,
 * k, |F_l|] optional. */
int oracle_hype_select(const float *objs, int64_t N, int M, const float *vref, const float *U,
                       int64_t s, int64_t n, int32_t *selected, double *d_out, int32_t *rank_out,
                       int64_t *info4)
{
    if (!objs || !vref || !U || !selected || N < 1 || M < 2 || M > 16 || s < 1 || n < 1 || n > N)
        return -1;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    double *hv = (double *)malloc(sizeof(double) * (size_t)N);
    hkey_t *last = (hkey_t *)malloc(sizeof(hkey_t) * (size_t)N);
    uint8_t *pick = (uint8_t *)calloc((size_t)N, 1);
    int rc = 0;
    if (!rank || !hv || !last || !pick) { rc = -1; goto done; }
    int32_t L = 0, l = 0;
    int64_t nb = 0, nl = 0;
    rc = oracle_ranks(objs, N, M, rank, &L);
    if (rc) goto done;
    rc = oracle_last_front(rank, N, n, &l, &nb, &nl);
    if (rc) goto done;
    const int64_t k = nb + nl - n;     /* |S| - n */
    rc = oracle_hype_hv(objs, N, M, vref, U, s, k, hv, NULL);
    if (rc) goto done;
    int64_t m = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] < l) pick[i] = 1;
        else if (rank[i] == l) { last[m].d = hv[i]; last[m].i = i; ++m; }
    }
    qsort(last, (size_t)m, sizeof(hkey_t), cmp_hkey);
    for (int64_t q = 0; q < n - nb; ++q) pick[last[q].i] = 1;
    int64_t t = 0;
    for (int64_t i = 0; i < N; ++i)
        if (pick[i]) selected[t++] = (int32_t)i;
    if (t != n) { rc = -1; goto done; }
    if (d_out) for (int64_t i = 0; i < N; ++i) d_out[i] = rank[i] <= l ? hv[i] : -INFINITY;
    if (rank_out) memcpy(rank_out, rank, sizeof(int32_t) * (size_t)N);
    if (info4) { info4[0] = l; info4[1] = L; info4[2] = k; info4[3] = nl; }
done:
    free(rank); free(hv); free(last); free(pick);
    return rc;
}
