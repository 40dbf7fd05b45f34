/*
 * Sanitizer driver for the CPU oracle (test infrastructure): runs every
 * oracle entry point on small seeded problems, including ties, duplicate rows,
 * the one-point and K = N cases and rejected arguments, and checks the
 * invariants that hold for any input.  Built with AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_sanitize.py; any out-of-bounds
 * access, leak or undefined operation aborts it.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_select_mode(const float *objs, int64_t N, int M, const float *refs, int H, int64_t K,
                       int niching, int32_t *selected, int32_t *rank_out, int32_t *niche_out,
                       double *dist_out, int32_t *dom_in, int32_t *dom_out, int64_t *info6);
int oracle_dominance_one(const float *objs, int64_t N, int M, int64_t j, int32_t *din,
                         int32_t *dout);
int oracle_rvea_gamma(const float *refs, int H, int M, double *gamma);
int oracle_rvea_select(const float *objs, int64_t N, int M, const float *refs, int H, int64_t t,
                       int64_t t_max, double alpha, int32_t *elite, int32_t *assign, double *apd,
                       double *theta, double *gap);
int oracle_hype_select(const float *objs, int64_t N, int M, const float *vref, const float *U,
                       int64_t s, int64_t n, int32_t *selected, double *d_out, int32_t *rank_out,
                       int64_t *info4);
int oracle_sbx_pm(const float *X, int64_t n, int d, const float *lower, const float *upper,
                  double eta_c, double eta_m, const float *r_sbx, const float *r_pm, double *out);
int oracle_gather_rows(const float *X, int64_t N, int d, const int32_t *idx, int64_t K,
                       float *out);

static uint64_t st = 0x9e3779b97f4a7c15ull;
static double unif(void)  /* xorshift64*, [0, 1) */
{
    st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
    return (double)((st * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

static int fails = 0;
#define CHECK(c) do { if (!(c)) { fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); ++fails; } } while (0)

static void fill_objs(float *f, int64_t N, int M, int quant)
{
    for (int64_t i = 0; i < N * M; ++i) {
        double v = unif();
        if (quant) v = floor(v * quant) / quant;
        f[i] = (float)v;
    }
}

static void one_selection(int64_t N, int M, int H, int64_t K, int quant, int niching)
{
    float *f = malloc(sizeof(float) * N * M), *r = malloc(sizeof(float) * H * M);
    int32_t *sel = malloc(sizeof(int32_t) * K), *rank = malloc(sizeof(int32_t) * N);
    int32_t *niche = malloc(sizeof(int32_t) * N), *din = malloc(sizeof(int32_t) * N);
    int32_t *dout = malloc(sizeof(int32_t) * N);
    double *dist = malloc(sizeof(double) * N);
    int64_t info[6];
    fill_objs(f, N, M, quant);
    if (N > 3) for (int k = 0; k < M; ++k) f[(N - 1) * M + k] = f[k];  /* a duplicate row */
    for (int j = 0; j < H * M; ++j) r[j] = (float)(0.05 + unif());
    int rc = oracle_select_mode(f, N, M, r, H, K, niching, sel, rank, niche, dist, din, dout, info);
    CHECK(rc == 0);
    if (rc == 0) {
        int64_t sum_in = 0, sum_out = 0;
        for (int64_t i = 0; i < N; ++i) { sum_in += din[i]; sum_out += dout[i]; }
        CHECK(sum_in == sum_out);
        for (int64_t q = 1; q < K; ++q) CHECK(sel[q - 1] < sel[q]);
        for (int64_t q = 0; q < K; ++q) CHECK(sel[q] >= 0 && sel[q] < N && rank[sel[q]] <= info[0]);
        for (int64_t i = 0; i < N; ++i) CHECK((rank[i] == 0) == (din[i] == 0));
        int32_t a = -1, b = -1;
        CHECK(oracle_dominance_one(f, N, M, N / 2, &a, &b) == 0);
        CHECK(a == din[N / 2] && b == dout[N / 2]);
    }
    free(f); free(r); free(sel); free(rank); free(niche); free(din); free(dout); free(dist);
}

int main(void)
{
    one_selection(300, 3, 20, 150, 0, 0);
    one_selection(300, 3, 20, 150, 16, 1);   /* many ties, one-shot niching */
    one_selection(257, 5, 35, 257, 8, 0);    /* K = N */
    one_selection(1, 2, 3, 1, 0, 0);         /* one point */
    one_selection(64, 16, 10, 7, 4, 0);      /* M = 16 */
    {   /* rejected arguments */
        float f[6] = {0, 1, 1, 0, 0.5f, 0.5f}, r[4] = {1, 0, 0, 1};
        int32_t sel[3];
        CHECK(oracle_select_mode(f, 3, 2, r, 2, 4, 0, sel, 0, 0, 0, 0, 0, 0) != 0);  /* K > N */
        CHECK(oracle_select_mode(f, 3, 1, r, 2, 1, 0, sel, 0, 0, 0, 0, 0, 0) != 0);  /* M = 1 */
        f[2] = NAN;
        CHECK(oracle_select_mode(f, 3, 2, r, 2, 1, 0, sel, 0, 0, 0, 0, 0, 0) != 0);  /* NaN */
    }
    {   /* RVEA */
        const int64_t N = 120; const int M = 3, H = 15;
        float *f = malloc(sizeof(float) * N * M), *r = malloc(sizeof(float) * H * M);
        int32_t *elite = malloc(sizeof(int32_t) * H), *assign = malloc(sizeof(int32_t) * N);
        double *apd = malloc(sizeof(double) * N), *theta = malloc(sizeof(double) * N);
        double *gap = malloc(sizeof(double) * N), gam[15];
        fill_objs(f, N, M, 0);
        for (int j = 0; j < H * M; ++j) r[j] = (float)(0.05 + unif());
        CHECK(oracle_rvea_gamma(r, H, M, gam) == 0);
        CHECK(oracle_rvea_select(f, N, M, r, H, 3, 10, 2.0, elite, assign, apd, theta, gap) == 0);
        for (int j = 0; j < H; ++j) CHECK(elite[j] < 0 || (elite[j] < N && assign[elite[j]] == j));
        free(f); free(r); free(elite); free(assign); free(apd); free(theta); free(gap);
    }
    {   /* HypE */
        const int64_t N = 80, s = 300, n = 40; const int M = 3;
        float *f = malloc(sizeof(float) * N * M), *U = malloc(sizeof(float) * s * M), vref[3];
        int32_t *sel = malloc(sizeof(int32_t) * n), *rank = malloc(sizeof(int32_t) * N);
        double *d = malloc(sizeof(double) * N);
        int64_t info[4];
        fill_objs(f, N, M, 8);
        for (int64_t q = 0; q < s * M; ++q) U[q] = (float)unif();
        for (int k = 0; k < M; ++k) vref[k] = 1.2f;
        CHECK(oracle_hype_select(f, N, M, vref, U, s, n, sel, d, rank, info) == 0);
        for (int64_t q = 1; q < n; ++q) CHECK(sel[q - 1] < sel[q]);
        free(f); free(U); free(sel); free(rank); free(d);
    }
    {   /* SBX + polynomial mutation, gather */
        const int64_t n = 11; const int d = 6;
        float *X = malloc(sizeof(float) * n * d), lo[6], hi[6];
        float *r1 = malloc(sizeof(float) * n * d), *r2 = malloc(sizeof(float) * n * d);
        double *out = malloc(sizeof(double) * n * d);
        for (int k = 0; k < d; ++k) { lo[k] = -1.0f; hi[k] = 2.0f; }
        for (int64_t q = 0; q < n * d; ++q) {
            X[q] = (float)(-1.0 + 3.0 * unif()); r1[q] = (float)unif(); r2[q] = (float)unif();
        }
        r1[0] = 0.0f; r2[1] = 0.0f; r2[2] = 0.5f;  /* closed-form draws */
        CHECK(oracle_sbx_pm(X, n, d, lo, hi, 15.0, 20.0, r1, r2, out) == 0);
        for (int64_t q = 0; q < (n / 2) * 2 * d; ++q) CHECK(out[q] >= -1.0 && out[q] <= 2.0);
        int32_t idx[4] = {10, 0, 3, 3};
        float *g = malloc(sizeof(float) * 4 * d);
        CHECK(oracle_gather_rows(X, n, d, idx, 4, g) == 0);
        CHECK(g[0] == X[10 * d] && g[2 * d + 1] == X[3 * d + 1]);
        idx[1] = (int32_t)n;  /* out of range */
        CHECK(oracle_gather_rows(X, n, d, idx, 4, g) != 0);
        free(X); free(r1); free(r2); free(out); free(g);
    }
    if (fails) { fprintf(stderr, "%d checks failed\n", fails); return 1; }
    printf("oracle sanitizer driver: ok\n");
    return 0;
}
