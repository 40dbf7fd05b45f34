/*
 * CPU oracle for NSGA-III environmental selection -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, float64 implementation of what the selection computes, used
 * to check the GPU library.  It shares no code with the GPU path.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it; the product path never does.
 *
 * Paper: "Bridging Evolutionary Multiobjective Optimization and GPU
 * Acceleration via Tensorization" (Liang et al., IEEE TEVC 2025).
 *
 * Stages (each function cites the passage it follows):
 *   oracle_dominance   Pareto dominance (Listing 1, Eq. (6)), in/out degree (Eq. (7))
 *   oracle_ranks       nondominated front of every point (Eq. (8)-(9), Alg. S.3)
 *   oracle_last_front  last admitted front l (Sec. IV-A.1, last step of Alg. S.3)
 *   oracle_normalize   ideal point, extreme points, intercepts (Alg. S.5)
 *   oracle_associate   perpendicular distance to reference lines (Eq. (10))
 *   oracle_niche_count niche counts over admitted fronts (Eq. (11))
 *   oracle_niching     niche-preserving pick from the last front (Alg. S.1)
 *   oracle_niching_oneshot  the one-shot niche selection (Sec. IV-A.5, Alg. S.4, Alg. S.6)
 *   oracle_select      the whole environmental selection (Alg. S.1 / S.4 outputs, Eq. (13))
 *
 * Readings of points the paper leaves open are fixed here and listed in the
 * design notes:
 *   - c counts the dominators of each point (the in-degree); only that makes
 *     p = 1{c = 0} the non-dominated set and matches the decrement sum_i p_i D_ij.
 *   - ranks are 0-based: front 0 holds the points nothing dominates.
 *   - l is the rank of the K-th smallest rank (0-based position K-1).
 *   - S = {r <= l}; the ideal point is taken over S.
 *   - extreme points use the achievement scalarising function with weight 1 on
 *     the own axis and 1e-6 elsewhere, realised as multiplication by 1e6;
 *     ties go to the lowest index.
 *   - intercepts: hyperplane through the translated extreme points (E b = 1,
 *     Gaussian elimination with partial pivoting, no fused multiply-add),
 *     rejected when a pivot is <= 1e-10 * max|E| or some b_k is not finite and
 *     positive or 1/b_k is not finite; then the nadir max_{S} (f - z); an
 *     intercept of 0 becomes 1.
 *   - distance: the residual form ||f' - (f'.rhat) rhat|| of the perpendicular
 *     distance (algebraically equal to Eq. (10)); argmin ties -> lowest index.
 *   - niche counts rho are taken over r < l (the members already admitted).
 *   - the "random" member of a crowded niche is the closest not yet chosen
 *     member by (distance, index).
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -fopenmp -shared -fPIC.
 * All int return codes: 0 ok, -1 invalid argument, -2 non-finite input.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENONFINITE (-2)

/* ------------------------------------------------------------------------ */
/* Pareto dominance, Listing 1 / Eq. (6): i dominates j iff f_i <= f_j in     */
/* every objective and f_i < f_j in at least one (minimisation, Eq. (1)).     */
/* ------------------------------------------------------------------------ */
static int dominates(const float *objs, int M, int64_t i, int64_t j)
{
    int all_le = 1, any_lt = 0;
    for (int k = 0; k < M; ++k) {
        double a = (double)objs[i * M + k];
        double b = (double)objs[j * M + k];
        if (!(a <= b)) all_le = 0;
        if (a < b) any_lt = 1;
    }
    return all_le && any_lt;
}

int oracle_dominates(const float *objs, int M, int64_t i, int64_t j)
{
    return dominates(objs, M, i, j);
}

static int check_finite(const float *a, int64_t n)
{
    for (int64_t t = 0; t < n; ++t)
        if (!isfinite(a[t])) return 0;
    return 1;
}

/* Eq. (7) read as the in-degree: dom_in[j] = #{i : D_ij}; also the out-degree
 * dom_out[i] = #{j : D_ij} (the paper's literal row sum). */
int oracle_dominance(const float *objs, int64_t N, int M, int32_t *dom_in, int32_t *dom_out)
{
    if (!objs || N < 1 || M < 1) return OR_EINVAL;
    if (!check_finite(objs, N * M)) return OR_ENONFINITE;
    #pragma omp parallel for schedule(dynamic, 64)
    for (int64_t j = 0; j < N; ++j) {
        int32_t cin = 0, cout = 0;
        for (int64_t i = 0; i < N; ++i) {
            if (i == j) continue;
            if (dominates(objs, M, i, j)) ++cin;
            if (dominates(objs, M, j, i)) ++cout;
        }
        if (dom_in) dom_in[j] = cin;
        if (dom_out) dom_out[j] = cout;
    }
    return OR_OK;
}

/* Dominance count of a single point (used for sampled checks at large N). */
int oracle_dominance_one(const float *objs, int64_t N, int M, int64_t j,
                         int32_t *dom_in_j, int32_t *dom_out_j)
{
    if (!objs || N < 1 || M < 1 || j < 0 || j >= N) return OR_EINVAL;
    int32_t cin = 0, cout = 0;
    for (int64_t i = 0; i < N; ++i) {
        if (i == j) continue;
        if (dominates(objs, M, i, j)) ++cin;
        if (dominates(objs, M, j, i)) ++cout;
    }
    *dom_in_j = cin;
    *dom_out_j = cout;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Nondominated fronts, Eq. (8)-(9) and Alg. S.3.                            */
/* The peeling of Eq. (8)-(9) puts a point in front k exactly when all of its */
/* dominators lie in fronts below k and one of them in front k-1, so          */
/*   rank[j] = 0                          if nothing dominates j,             */
/*   rank[j] = 1 + max{rank[i] : i dom j}  otherwise                          */
/* (the length of the longest dominance chain ending at j).  That recursion   */
/* is evaluated here directly, visiting the points in an order in which every */
/* dominator comes first: ascending float64 sum of the objectives, then       */
/* lexicographic objectives, then index.  If i dominates j, each term of i's  */
/* sum is <= j's and rounding is monotone, so sum_i <= sum_j; with equal sums */
/* the first objective where the two differ is smaller for i.                 */
/* ------------------------------------------------------------------------ */
typedef struct { double sum; int64_t i; const float *row; int M; } order_key_t;

static int cmp_order(const void *pa, const void *pb)
{
    const order_key_t *a = (const order_key_t *)pa, *b = (const order_key_t *)pb;
    if (a->sum < b->sum) return -1;
    if (a->sum > b->sum) return 1;
    for (int k = 0; k < a->M; ++k) {
        double x = (double)a->row[k], y = (double)b->row[k];
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

int oracle_ranks(const float *objs, int64_t N, int M, int32_t *rank, int32_t *num_fronts)
{
    if (!objs || !rank || N < 1 || M < 1) return OR_EINVAL;
    if (!check_finite(objs, N * M)) return OR_ENONFINITE;
    order_key_t *ord = (order_key_t *)malloc(sizeof(order_key_t) * (size_t)N);
    if (!ord) return OR_EINVAL;
    for (int64_t i = 0; i < N; ++i) {
        double s = 0.0;
        for (int k = 0; k < M; ++k) s = s + (double)objs[i * M + k];
        ord[i].sum = s;
        ord[i].i = i;
        ord[i].row = objs + i * M;
        ord[i].M = M;
    }
    qsort(ord, (size_t)N, sizeof(order_key_t), cmp_order);
    int32_t L = 0;
    for (int64_t t = 0; t < N; ++t) {
        const int64_t j = ord[t].i;
        int32_t best = -1;   /* highest rank among the dominators of j seen so far */
        #pragma omp parallel for schedule(static) reduction(max : best) if (t > 4096)
        for (int64_t u = 0; u < t; ++u) {
            const int64_t i = ord[u].i;
            if (dominates(objs, M, i, j) && rank[i] > best) best = rank[i];
        }
        rank[j] = best + 1;
        if (rank[j] + 1 > L) L = rank[j] + 1;
    }
    if (num_fronts) *num_fronts = L;
    free(ord);
    return OR_OK;
}

/* l = sort(r)[K-1] (Sec. IV-A.1 end; Alg. S.3 last step, 0-based position). */
int oracle_last_front(const int32_t *rank, int64_t N, int64_t K,
                      int32_t *l_out, int64_t *n_before, int64_t *n_last)
{
    if (!rank || N < 1 || K < 1 || K > N) return OR_EINVAL;
    int32_t maxr = 0;
    for (int64_t i = 0; i < N; ++i) if (rank[i] > maxr) maxr = rank[i];
    int64_t *hist = (int64_t *)calloc((size_t)maxr + 1, sizeof(int64_t));
    if (!hist) return OR_EINVAL;
    for (int64_t i = 0; i < N; ++i) hist[rank[i]]++;
    int64_t cum = 0;
    int32_t l = 0;
    for (int32_t r = 0; r <= maxr; ++r) {
        if (cum + hist[r] >= K) { l = r; break; }
        cum += hist[r];
    }
    if (l_out) *l_out = l;
    if (n_before) *n_before = cum;
    if (n_last) *n_last = hist[l];
    free(hist);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Normalisation, Alg. S.5, over S = {r <= l}.                                */
/* Outputs: z[M] ideal point, a[M] intercepts, extreme[M] point indices,      */
/* *fallback: 0 hyperplane intercepts, 1 nadir, 2 nadir with a zero replaced. */
/* ------------------------------------------------------------------------ */
int oracle_normalize(const float *objs, int64_t N, int M, const int32_t *rank, int32_t l,
                     double *z, double *a, int32_t *extreme, int32_t *fallback)
{
    if (!objs || !rank || !z || !a || N < 1 || M < 1 || M > 64) return OR_EINVAL;
    /* ideal point z = min_{i in S} f_i */
    for (int k = 0; k < M; ++k) z[k] = INFINITY;
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] > l) continue;
        for (int k = 0; k < M; ++k) {
            double v = (double)objs[i * M + k];
            if (v < z[k]) z[k] = v;
        }
    }
    /* extreme points: e_j = argmin_{i in S} max_k (f_ik - z_k) * w_jk,
     * w_jj = 1, w_jk = 1e6 for k != j (the 1/eps weights) */
    double E[64 * 64];
    double nadir[64];
    int32_t ext[64];
    for (int k = 0; k < M; ++k) nadir[k] = 0.0;
    for (int j = 0; j < M; ++j) {
        double best = INFINITY;
        int64_t bi = -1;
        for (int64_t i = 0; i < N; ++i) {
            if (rank[i] > l) continue;
            double asf = -INFINITY;
            for (int k = 0; k < M; ++k) {
                double g = (double)objs[i * M + k] - z[k];
                double v = (k == j) ? g : g * 1e6;
                if (v > asf) asf = v;
            }
            if (asf < best) { best = asf; bi = i; }
        }
        ext[j] = (int32_t)bi;
        for (int k = 0; k < M; ++k) E[j * M + k] = (double)objs[bi * M + k] - z[k];
    }
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] > l) continue;
        for (int k = 0; k < M; ++k) {
            double g = (double)objs[i * M + k] - z[k];
            if (g > nadir[k]) nadir[k] = g;
        }
    }
    if (extreme) for (int j = 0; j < M; ++j) extreme[j] = ext[j];

    /* intercepts: solve E b = 1; a_k = 1 / b_k */
    double A[64 * 64], rhs[64], b[64];
    double maxabs = 0.0;
    for (int t = 0; t < M * M; ++t) {
        A[t] = E[t];
        double v = fabs(E[t]);
        if (v > maxabs) maxabs = v;
    }
    for (int k = 0; k < M; ++k) rhs[k] = 1.0;
    int ok = maxabs > 0.0;
    for (int c = 0; c < M && ok; ++c) {
        int p = c;
        double pv = fabs(A[c * M + c]);
        for (int r = c + 1; r < M; ++r) {
            double v = fabs(A[r * M + c]);
            if (v > pv) { pv = v; p = r; }
        }
        if (!(pv > 1e-10 * maxabs)) { ok = 0; break; }
        if (p != c) {
            for (int k = 0; k < M; ++k) { double t = A[c * M + k]; A[c * M + k] = A[p * M + k]; A[p * M + k] = t; }
            double t = rhs[c]; rhs[c] = rhs[p]; rhs[p] = t;
        }
        for (int r = c + 1; r < M; ++r) {
            double f = A[r * M + c] / A[c * M + c];
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
            if (!(isfinite(b[k]) && b[k] > 0.0)) { ok = 0; break; }
            double ak = 1.0 / b[k];
            if (!isfinite(ak)) { ok = 0; break; }
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
    if (fallback) *fallback = fb;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Association, Eq. (10): normalised point f' = (f - z) / a, distance to the  */
/* line through reference direction R_j, residual form                        */
/*   s = f' . rhat_j,  d_ij = || f' - s rhat_j ||,  rhat_j = R_j / ||R_j||.   */
/* pi_i = argmin_j d_ij (lowest j on ties), d_i = min_j d_ij, for i in S;     */
/* -1 elsewhere.  gap[i] = (d2 - d1) / max(d2, 1e-300) for the two smallest.  */
/* ------------------------------------------------------------------------ */
int oracle_associate(const float *objs, int64_t N, int M, const int32_t *rank, int32_t l,
                     const double *z, const double *a, const float *refs, int H,
                     int32_t *niche, double *dist, double *gap)
{
    if (!objs || !rank || !z || !a || !refs || !niche || N < 1 || M < 1 || M > 64 || H < 1)
        return OR_EINVAL;
    if (!check_finite(refs, (int64_t)H * M)) return OR_ENONFINITE;
    double *rhat = (double *)malloc(sizeof(double) * (size_t)H * M);
    if (!rhat) return OR_EINVAL;
    for (int j = 0; j < H; ++j) {
        double nn = 0.0;
        for (int k = 0; k < M; ++k) {
            double v = (double)refs[j * M + k];
            if (v < 0.0) { free(rhat); return OR_ENONFINITE; }
            nn = nn + v * v;
        }
        double n = sqrt(nn);
        if (!(n > 0.0)) { free(rhat); return OR_ENONFINITE; }
        for (int k = 0; k < M; ++k) rhat[j * M + k] = (double)refs[j * M + k] / n;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] > l) {
            niche[i] = -1;
            if (dist) dist[i] = -1.0;
            if (gap) gap[i] = -1.0;
            continue;
        }
        double fp[64];
        for (int k = 0; k < M; ++k) fp[k] = ((double)objs[i * M + k] - z[k]) / a[k];
        double d1 = INFINITY, d2 = INFINITY;
        int32_t best = -1;
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int k = 0; k < M; ++k) s = s + fp[k] * rhat[j * M + k];
            double q = 0.0;
            for (int k = 0; k < M; ++k) {
                double e = fp[k] - s * rhat[j * M + k];
                q = q + e * e;
            }
            double d = sqrt(q);
            if (d < d1) { d2 = d1; d1 = d; best = j; }
            else if (d < d2) { d2 = d; }
        }
        niche[i] = best;
        if (dist) dist[i] = d1;
        if (gap) gap[i] = (H > 1) ? (d2 - d1) / fmax(d2, 1e-300) : INFINITY;
    }
    free(rhat);
    return OR_OK;
}

/* Niche counts, Eq. (11) over the admitted members r < l. */
int oracle_niche_count(const int32_t *rank, const int32_t *niche, int64_t N, int32_t l,
                       int H, int32_t *rho)
{
    if (!rank || !niche || !rho || N < 1 || H < 1) return OR_EINVAL;
    for (int j = 0; j < H; ++j) rho[j] = 0;
    for (int64_t i = 0; i < N; ++i)
        if (rank[i] < l) {
            if (niche[i] < 0 || niche[i] >= H) return OR_EINVAL;
            rho[niche[i]]++;
        }
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Niche-preserving pick from the last front, Alg. S.1.                       */
/* The rule: R members of F_l are admitted one at a time.  Each admission     */
/* goes to the reference with the smallest niche count rho_j among those that */
/* still have unadmitted F_l members associated with them (lowest j on ties); */
/* that reference admits its closest such member (smallest distance, then     */
/* lowest index -- one of the outcomes the paper's random choice allows) and  */
/* its niche count grows by one.  chosen[i] = 1 for the admitted members.     */
/* ------------------------------------------------------------------------ */
typedef struct { double d; int64_t i; } dkey_t;

static int cmp_dkey(const void *pa, const void *pb)
{
    const dkey_t *a = (const dkey_t *)pa, *b = (const dkey_t *)pb;
    if (a->d < b->d) return -1;
    if (a->d > b->d) return 1;
    return (a->i < b->i) ? -1 : (a->i > b->i);
}

/* Members of F_l grouped by reference, each group in (distance, index) order:
 * group j occupies cand[first[j] .. first[j+1]).  Returns |F_l|, or -1 when a
 * member's reference is out of range or memory runs out. */
static int64_t group_last_front(const int32_t *rank, const int32_t *niche, const double *dist,
                                int64_t N, int32_t l, int H, dkey_t **cand_out, int64_t **first_out)
{
    int64_t *first = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    int64_t *fill = (int64_t *)calloc((size_t)H, sizeof(int64_t));
    int64_t nl = 0;
    if (!first || !fill) { free(first); free(fill); return -1; }
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] != l) continue;
        if (niche[i] < 0 || niche[i] >= H) { free(first); free(fill); return -1; }
        first[niche[i] + 1]++;
        ++nl;
    }
    for (int j = 0; j < H; ++j) first[j + 1] += first[j];
    dkey_t *cand = (dkey_t *)malloc(sizeof(dkey_t) * (size_t)(nl > 0 ? nl : 1));
    if (!cand) { free(first); free(fill); return -1; }
    for (int64_t i = 0; i < N; ++i) {
        if (rank[i] != l) continue;
        dkey_t *c = &cand[first[niche[i]] + fill[niche[i]]++];
        c->d = dist[i];
        c->i = i;
    }
    for (int j = 0; j < H; ++j)
        qsort(cand + first[j], (size_t)(first[j + 1] - first[j]), sizeof(dkey_t), cmp_dkey);
    free(fill);
    *cand_out = cand;
    *first_out = first;
    return nl;
}

int oracle_niching(const int32_t *rank, const int32_t *niche, const double *dist, int64_t N,
                   int32_t l, int H, int64_t R, const int32_t *rho_in, uint8_t *chosen)
{
    if (!rank || !niche || !dist || !rho_in || !chosen || N < 1 || H < 1 || R < 0) return OR_EINVAL;
    dkey_t *cand = NULL;
    int64_t *first = NULL;
    const int64_t nl = group_last_front(rank, niche, dist, N, l, H, &cand, &first);
    if (nl < 0) return OR_EINVAL;
    int64_t *used = (int64_t *)calloc((size_t)H, sizeof(int64_t));  /* admitted per reference */
    int64_t *rho = (int64_t *)malloc(sizeof(int64_t) * (size_t)H);
    if (!used || !rho || R > nl) { free(cand); free(first); free(used); free(rho); return OR_EINVAL; }
    for (int j = 0; j < H; ++j) rho[j] = rho_in[j];
    memset(chosen, 0, (size_t)N);
    for (int64_t admitted = 0; admitted < R; ++admitted) {
        int jmin = -1;
        for (int j = 0; j < H; ++j) {
            const int has_members = used[j] < first[j + 1] - first[j];
            if (has_members && (jmin < 0 || rho[j] < rho[jmin])) jmin = j;
        }
        /* R <= |F_l| guarantees some reference still has members */
        chosen[cand[first[jmin] + used[jmin]].i] = 1;
        used[jmin]++;
        rho[jmin]++;
    }
    free(cand); free(first); free(used); free(rho);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* One-shot niche selection of the tensorized algorithm (Sec. IV-A.5; the     */
/* niche-selection steps of Alg. S.4 and Alg. S.6), which the paper offers as */
/* a parallel approximation of the loop above.  Reading of its steps:         */
/*   E = references with rho_j = 0 (no admitted member) that have at least   */
/*       one F_l member (the others are masked with infinity);               */
/*   every j in E picks its closest F_l member (smallest distance, lowest    */
/*       index on ties: the argmin over the match matrix);                   */
/*   n_dif = R - |E|;                                                         */
/*   n_dif > 0: the n_dif lowest-index unpicked F_l members are added        */
/*       (the ascending sort of the remaining last-front indices);           */
/*   n_dif < 0: the |n_dif| picks with the highest indices are dropped, i.e. */
/*       the R lowest-index picks are kept.                                  */
/* On the shuffled population the algorithm takes as input, index order is a */
/* random order, so both fill rules are the paper's random choices.           */
/* chosen[i] = 1 for the R admitted members; *n_empty (optional) = |E|.       */
/* ------------------------------------------------------------------------ */
int oracle_niching_oneshot(const int32_t *rank, const int32_t *niche, const double *dist,
                           int64_t N, int32_t l, int H, int64_t R, const int32_t *rho_in,
                           uint8_t *chosen, int64_t *n_empty)
{
    if (!rank || !niche || !dist || !rho_in || !chosen || N < 1 || H < 1 || R < 0) return OR_EINVAL;
    dkey_t *cand = NULL;
    int64_t *first = NULL;
    const int64_t nl = group_last_front(rank, niche, dist, N, l, H, &cand, &first);
    if (nl < 0) return OR_EINVAL;
    if (R > nl) { free(cand); free(first); return OR_EINVAL; }
    memset(chosen, 0, (size_t)N);
    int64_t ne = 0;
    for (int j = 0; j < H; ++j)
        if (rho_in[j] == 0 && first[j + 1] > first[j]) {
            chosen[cand[first[j]].i] = 1;          /* closest member of an empty niche */
            ++ne;
        }
    int64_t ndif = R - ne;
    if (ndif > 0) {
        for (int64_t i = 0; i < N && ndif > 0; ++i)
            if (rank[i] == l && !chosen[i]) { chosen[i] = 1; --ndif; }
    } else if (ndif < 0) {
        for (int64_t i = N - 1; i >= 0 && ndif < 0; --i)
            if (chosen[i]) { chosen[i] = 0; ++ndif; }
    }
    if (n_empty) *n_empty = ne;
    free(cand); free(first);
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Whole selection (Alg. S.1, outputs as Eq. (13): ascending indices).        */
/* niching: 0 the loop of Alg. S.1, 1 the one-shot form of Alg. S.4.         */
/* Outputs may be NULL except selected.  info6 (optional):                   */
/* [l, num_fronts, |F_l|, R, fallback, near_ties (gap < 1e-6)].               */
/* ------------------------------------------------------------------------ */
int oracle_select_mode(const float *objs, int64_t N, int M, const float *refs, int H, int64_t K,
                       int niching, int32_t *selected, int32_t *rank_out, int32_t *niche_out,
                       double *dist_out, int32_t *dom_in, int32_t *dom_out, int64_t *info6)
{
    if (niching != 0 && niching != 1) return OR_EINVAL;
    if (!objs || !refs || !selected || N < 1 || M < 2 || M > 16 || H < 1 || H > 65535 ||
        K < 1 || K > N || N > 2147483647LL)
        return OR_EINVAL;
    if (!check_finite(objs, N * M) || !check_finite(refs, (int64_t)H * M)) return OR_ENONFINITE;
    int rc = OR_OK;
    int32_t *rank = (int32_t *)malloc(sizeof(int32_t) * N);
    int32_t *niche = (int32_t *)malloc(sizeof(int32_t) * N);
    double *dist = (double *)malloc(sizeof(double) * N);
    double *gap = (double *)malloc(sizeof(double) * N);
    int32_t *rho = (int32_t *)malloc(sizeof(int32_t) * H);
    uint8_t *chosen = (uint8_t *)malloc((size_t)N);
    if (!rank || !niche || !dist || !gap || !rho || !chosen) { rc = OR_EINVAL; goto done; }

    if (dom_in || dom_out) {
        rc = oracle_dominance(objs, N, M, dom_in, dom_out);
        if (rc) goto done;
    }
    int32_t L = 0;
    rc = oracle_ranks(objs, N, M, rank, &L);
    if (rc) goto done;
    int32_t l;
    int64_t nb, nl;
    rc = oracle_last_front(rank, N, K, &l, &nb, &nl);
    if (rc) goto done;
    double z[64], a[64];
    int32_t fb = 0;
    rc = oracle_normalize(objs, N, M, rank, l, z, a, NULL, &fb);
    if (rc) goto done;
    rc = oracle_associate(objs, N, M, rank, l, z, a, refs, H, niche, dist, gap);
    if (rc) goto done;
    rc = oracle_niche_count(rank, niche, N, l, H, rho);
    if (rc) goto done;
    if (niching == 0)
        rc = oracle_niching(rank, niche, dist, N, l, H, K - nb, rho, chosen);
    else
        rc = oracle_niching_oneshot(rank, niche, dist, N, l, H, K - nb, rho, chosen, NULL);
    if (rc) goto done;
    int64_t t = 0;
    for (int64_t i = 0; i < N; ++i)
        if (rank[i] < l || chosen[i]) selected[t++] = (int32_t)i;
    if (t != K) { rc = OR_EINVAL; goto done; }
    int64_t nt = 0;
    for (int64_t i = 0; i < N; ++i)
        if (rank[i] <= l && gap[i] < 1e-6) ++nt;
    if (rank_out) memcpy(rank_out, rank, sizeof(int32_t) * N);
    if (niche_out) memcpy(niche_out, niche, sizeof(int32_t) * N);
    if (dist_out) memcpy(dist_out, dist, sizeof(double) * N);
    if (info6) {
        info6[0] = l; info6[1] = L; info6[2] = nl; info6[3] = K - nb; info6[4] = fb; info6[5] = nt;
    }
done:
    free(rank); free(niche); free(dist); free(gap); free(rho); free(chosen);
    return rc;
}

int oracle_select(const float *objs, int64_t N, int M, const float *refs, int H, int64_t K,
                  int32_t *selected, int32_t *rank_out, int32_t *niche_out, double *dist_out,
                  int32_t *dom_in, int32_t *dom_out, int64_t *info6)
{
    return oracle_select_mode(objs, N, M, refs, H, K, 0, selected, rank_out, niche_out, dist_out,
                              dom_in, dom_out, info6);
}

/* Thread count for later calls from this thread (timing of the one-thread
 * oracle); n < 1 restores one thread per host core. */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
#else
    (void)n;
#endif
}

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
