/*
 * nsga3.h -- NSGA-III environmental selection on one AMD Instinct MI355X (gfx950).
 *
 * The library computes the environmental selection of NSGA-III on a merged
 * population: Pareto-dominance counts and nondominated fronts, ideal/extreme
 * point normalisation, association of every admitted point with its closest
 * reference line, niche counts, and the niche-preserving pick from the last
 * admitted front.
 *
 * Paper: Liang, Li, Yu, Sun, Cheng, "Bridging Evolutionary Multiobjective
 * Optimization and GPU Acceleration via Tensorization", IEEE TEVC 2025.
 *   - selection as a whole: Sec. IV-A; Alg. S.1 (original) and Alg. S.4 (tensorized)
 *   - dominance: Listing 1, Eq. (6); dominance count: Eq. (7)
 *   - fronts: Eq. (8)-(9), Alg. S.3; last front l: end of Sec. IV-A.1
 *   - normalisation: Alg. S.5;  association: Eq. (10);  niche counts: Eq. (11)
 *   - niching: Alg. S.1 (its inner loop), or the one-shot form of Sec. IV-A.5
 *     (Alg. S.4, Alg. S.6);  output indices: Eq. (13)
 *
 * Conventions shared by all entry points
 *   - All objectives are minimised (Eq. (1)).  Objective matrices are N x M,
 *     row-major float32; reference matrices are H x M, row-major float32 with
 *     non-negative entries and a non-zero norm per row.
 *   - Pointers marked DEVICE are device memory on the context's device; every
 *     other pointer is host memory.  The caller owns every buffer it passes;
 *     the context owns its workspace.
 *   - Calls that take a stream are asynchronous and stream-ordered: outputs are
 *     valid once the stream has been synchronised.  No call synchronises the
 *     stream or the device unless stated.
 *   - Errors that can be checked on the host are returned immediately and
 *     nothing is enqueued.  Errors that need the data (non-finite values, a bad
 *     reference row) are reported through nsga3_info.status on the device; the
 *     outputs of such a call are then undefined.
 *   - A context is not thread-safe: use one context per host thread.  A context
 *     stays usable after any error.
 */
#ifndef NSGA3_H
#define NSGA3_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    NSGA3_OK = 0,
    NSGA3_E_INVALID = -1,      /* bad argument (null pointer, size out of range) */
    NSGA3_E_NONFINITE = -2,    /* NaN/Inf objective, or invalid reference row (device-side) */
    NSGA3_E_NOMEM = -3,        /* workspace allocation failed or exceeds the configured cap */
    NSGA3_E_HIP = -4,          /* a HIP runtime call failed */
    NSGA3_E_UNSUPPORTED = -5   /* device is not gfx950, or cooperative launch unavailable */
} nsga3_status;

typedef enum {
    NSGA3_ASSOC_FP32 = 0,      /* candidate screening in float32 on the vector ALUs */
    NSGA3_ASSOC_BF16 = 1       /* candidate screening in bfloat16 on the matrix cores */
} nsga3_assoc_mode;

typedef enum {
    NSGA3_NICHING_EXACT = 0,      /* the niche-preserving loop of Alg. S.1 (one member at a time:
                                     least-crowded reference first, its closest member) */
    NSGA3_NICHING_ONESHOT = 1     /* the one-shot tensorized form (Sec. IV-A.5; niche-selection
                                     steps of Alg. S.4, Alg. S.6): every reference with no admitted
                                     member and some last-front member admits its closest one at
                                     once; a shortfall is filled with the lowest-index remaining
                                     last-front members, a surplus keeps the lowest-index picks
                                     (index order is the random order of the shuffled population
                                     the paper takes as input).  An approximation of the loop. */
} nsga3_niching_mode;

typedef struct {
    nsga3_assoc_mode assoc;       /* default NSGA3_ASSOC_FP32 */
    int32_t autotune;             /* 1: nsga3_plan_create times candidate work-item shapes per
                                     (M, N range) on the plan's own problems and keeps the
                                     fastest (cached in the context); 0: fixed defaults.
                                     Results never depend on the choice. */
    size_t max_workspace_bytes;   /* 0 = no cap */
    nsga3_niching_mode niching;   /* default NSGA3_NICHING_EXACT.  Batched plans of a context with
                                     NSGA3_NICHING_ONESHOT run as a graph of single selections. */
} nsga3_options;

/* Per-call diagnostics, written on-stream into DEVICE memory. */
typedef struct {
    int32_t status;               /* NSGA3_OK or NSGA3_E_NONFINITE */
    int32_t last_front;           /* l: rank of the K-th smallest rank (0-based) */
    int32_t num_fronts;           /* L: number of nondominated fronts */
    int32_t last_front_size;      /* |F_l| */
    int32_t num_from_last;        /* R = K - #{rank < l}: members picked from F_l */
    int32_t intercept_fallback;   /* 0 hyperplane, 1 nadir, 2 nadir with a zero axis set to 1 */
    int32_t near_ties;            /* admitted points whose two closest reference lines among
                                     the candidates that survive screening are within 1e-6
                                     relative distance after float64 re-scoring.  A line
                                     screened out is never counted, so this is a lower bound
                                     on the number over all H lines (diagnostic only). */
    int32_t reserved;             /* device error bits of the last failing check (diagnostic;
                                     0 when status is NSGA3_OK) */
} nsga3_info;

typedef struct nsga3_ctx nsga3_ctx;

/* Create a context on HIP device `device` (must be gfx950).  `opt` may be NULL
 * for the defaults.  On success *out receives the context. */
nsga3_status nsga3_create(nsga3_ctx **out, int device, const nsga3_options *opt);

/* Destroy a context and free its workspace.  Waits for nothing: the caller must
 * make sure no work using the context is still running.  NULL is ignored. */
void nsga3_destroy(nsga3_ctx *ctx);

/* Grow the context's workspace so that later calls with N <= N_max, M <= M_max,
 * H <= H_max allocate nothing.  Synchronous (allocation).  Sizes are checked as
 * in nsga3_select. */
nsga3_status nsga3_reserve(nsga3_ctx *ctx, int64_t N_max, int32_t M_max, int32_t H_max);

/* Bytes of workspace a call of this size needs (host-only query). */
nsga3_status nsga3_workspace_size(int64_t N, int32_t M, int32_t H, size_t *bytes);

/*
 * Environmental selection of K out of N points (Alg. S.1 / Alg. S.4).
 *
 *   objs      DEVICE float[N*M]  objective values, row-major, minimised
 *   N         1 <= N <= 2^31-1   merged population size
 *   M         2 <= M <= 16       number of objectives
 *   refs      DEVICE float[H*M]  reference directions (rows >= 0, non-zero norm)
 *   H         1 <= H <= 65535    number of reference directions
 *   K         1 <= K <= N        number of points to select
 *   selected  DEVICE int32[K]    required: selected point indices, ascending (Eq. (13))
 *   rank      DEVICE int32[N]    optional: 0-based front index of every point (Eq. (8)-(9))
 *   niche     DEVICE int32[N]    optional: closest reference line for rank <= l, else -1 (Eq. (10))
 *   dist      DEVICE float[N]    optional: perpendicular distance to it (normalised
 *                                objective space, Alg. S.5), else -1
 *   dom_in    DEVICE int32[N]    optional: number of points dominating each point (Eq. (7))
 *   dom_out   DEVICE int32[N]    optional: number of points each point dominates
 *   info      DEVICE nsga3_info* optional: diagnostics (see nsga3_info)
 *   stream    HIP stream to enqueue on (0 = legacy default stream)
 *
 * Determinism: every output is a function of the inputs only (no dependence on
 * scheduling).  Ties are resolved by lowest index everywhere; the "random"
 * member of a crowded niche (Alg. S.1) is its closest remaining member.
 * Workspace grows on demand (synchronous allocation) unless nsga3_reserve was
 * called with sufficient sizes.
 */
nsga3_status nsga3_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                          const float *refs, int32_t H, int64_t K,
                          int32_t *selected, int32_t *rank, int32_t *niche, float *dist,
                          int32_t *dom_in, int32_t *dom_out, nsga3_info *info,
                          hipStream_t stream);

/*
 * Variation around the selection (Supplementary Sec. S.I): simulated binary
 * crossover (Eq. (S.6)-(S.7)) of rows r and h + r of the n x d population X
 * (h = floor(n / 2); children at rows r and h + r of `offspring`), the children
 * clipped to [lower, upper], then polynomial mutation (Eq. (S.8)-(S.11)) of
 * every variable of both children.  With a draw m per (row, variable):
 *   B = (2m)^(1/(eta_c+1)) for m <= 1/2, else (1/(2 - 2m))^(1/(eta_c+1));
 *   children ((1 +- B) x1 + (1 -+ B) x2) / 2;
 *   mutation step (eta = eta_m + 1, D = u - l, d1 = (x - l)/D, d2 = (u - x)/D):
 *   (2m + (1 - 2m)(1 - d1)^eta)^(1/eta) - 1 for m <= 1/2, else
 *   1 - (2 - 2m + (2m - 1)(1 - d2)^eta)^(1/eta); x' = x + step D.
 *
 *   X          DEVICE float[n*d]   population, row-major (n >= 2; an odd last row is unused)
 *   lower, upper DEVICE float[d]   bounds, finite, lower < upper
 *   eta_c, eta_m                   distribution indices (finite, >= 0)
 *   r_sbx      DEVICE float[h*d]   the caller's uniform draws in [0, 1) for the crossover
 *   r_pm       DEVICE float[2h*d]  ... and for the mutation of every child variable
 *   offspring  DEVICE float[2h*d]  output
 *   status     DEVICE int32*       optional: NSGA3_OK, or NSGA3_E_NONFINITE (bad bounds or a
 *                                  non-finite result)
 * Float32 arithmetic (powers through the hardware base-2 logarithm and
 * exponential).  Needs no context and allocates nothing.  Asynchronous.
 */
nsga3_status nsga3_sbx_pm(const float *X, int64_t n, int32_t d, const float *lower,
                          const float *upper, double eta_c, double eta_m, const float *r_sbx,
                          const float *r_pm, float *offspring, int32_t *status, hipStream_t stream);

/*
 * Gather of the selected rows (Eq. (13)): out row q = X row idx[q].
 *   X DEVICE float[N*d], idx DEVICE int32[K], out DEVICE float[K*d];
 *   status DEVICE int32* optional: NSGA3_E_INVALID if an index lies outside
 *   [0, N) (that row is not written).  Needs no context.  Asynchronous.
 */
nsga3_status nsga3_gather_rows(const float *X, int64_t N, int32_t d, const int32_t *idx, int64_t K,
                               float *out, int32_t *status, hipStream_t stream);

/*
 * Environmental selection of TensorHypE (Sec. IV-C; Supplementary Alg. S.10,
 * S.11): the nondominated sort of nsga3_select gives ranks r and the last
 * admitted front l for a population of n; every point of r < l is kept, and
 * the members of F_l with the largest Monte Carlo hypervolume estimates fill
 * the remaining places (lowest index among equal estimates).  Estimation
 * over all N points (as printed): k = |{r <= l}| - n,
 * alpha_c = (1/c) prod_{i=1}^{c-1} (k - i) / (N - i); f_l = the per-objective
 * minimum; sample i = f_l + U_i (vref - f_l), rounded to float32;
 * count_i = #{p : F_p <= sample i in every objective};
 * HV_p = V / s * sum over the samples p dominates with count_i <= k of
 * alpha_{count_i}, V = prod_j (vref_j - f_l,j).
 *
 *   objs      DEVICE float[N*M]  objective values, row-major, minimised (2 <= M <= 16)
 *   vref      DEVICE float[M]    reference point (the upper corner of the sampling box)
 *   U         DEVICE float[s*M]  the caller's uniform draws in [0, 1), row-major
 *   s         1 <= s <= 2^31-1   number of samples
 *   n         1 <= n <= N        population size to keep
 *   selected  DEVICE int32[n]    required: kept indices, ascending
 *   d         DEVICE double[N]   optional: HV estimate for rank <= l, -inf elsewhere
 *   rank      DEVICE int32[N]    optional: 0-based front index
 *   info      DEVICE nsga3_info* optional: status and front statistics
 * Host-checkable errors return NSGA3_E_INVALID and enqueue nothing; non-finite
 * objectives, draws or reference point set info.status = NSGA3_E_NONFINITE.
 * The estimates are float64; the alpha products are formed in chunks, so they
 * may differ from a sequential product in the last bits.  Uses the context's
 * workspace (grown on demand).  Asynchronous on `stream`.
 */
nsga3_status nsga3_hype_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                               const float *vref, const float *U, int64_t s, int64_t n,
                               int32_t *selected, double *d, int32_t *rank, nsga3_info *info,
                               hipStream_t stream);

/*
 * Environmental selection of TensorRVEA (Supplementary Sec. S.V, Alg. S.12):
 * one elite per reference vector by the angle-penalized distance.  With
 * z = the per-objective minimum over all N points and F' = F - z, every
 * point joins the partition of the reference with the smallest angle theta
 * to F' (the largest F'.V_j / ||V_j||, lowest j on ties); gamma_j is the
 * smallest angle between V_j and another reference;
 *   APD_i = (1 + M (t / t_max)^alpha theta_i / gamma_{a_i}) ||F'_i||
 * (the penalty factor computed on the host in float64); elite_j is the point
 * of partition j with the smallest APD (lowest index on ties), -1 when the
 * partition is empty.  A point equal to z joins partition 0 with APD 0.
 *
 *   objs    DEVICE float[N*M]  objective values, row-major, minimised
 *   N, M    1 <= N <= 2^31-1, 2 <= M <= 16
 *   refs    DEVICE float[H*M]  reference vectors (rows >= 0, non-zero, distinct
 *                              directions), 2 <= H <= 65535
 *   t, t_max, alpha            generation counter (t >= 0, t_max >= 1) and the rate of
 *                              change of the penalty (finite, >= 0)
 *   elite   DEVICE int32[H]    required: elite of every partition, or -1
 *   assign  DEVICE int32[N]    optional: partition of every point
 *   apd     DEVICE double[N]   optional: angle-penalized distance of every point
 *   info    DEVICE nsga3_info* optional: only status (and reserved) are set
 * Host-checkable errors return NSGA3_E_INVALID and enqueue nothing; a
 * non-finite objective, an invalid reference row or two references with the
 * same direction (gamma = 0) set info.status = NSGA3_E_NONFINITE on the
 * device, and elite is then undefined.  Uses the context's workspace (grown
 * on demand; nsga3_reserve does not size it).  Asynchronous on `stream`.
 */
nsga3_status nsga3_rvea_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                               const float *refs, int32_t H, int64_t t, int64_t t_max, double alpha,
                               int32_t *elite, int32_t *assign, double *apd, nsga3_info *info,
                               hipStream_t stream);

/*
 * Allocation-free form of nsga3_select, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, outputs and results as nsga3_select with
 * float32 association screening, on the current HIP device, without a
 * context.  The workspace is a fixed array of NSGA3_NOALLOC_MAX_WORKSPACE
 * bytes that every device holds for the life of the process; a call whose
 * workspace (nsga3_workspace_size) is larger returns NSGA3_E_NOMEM and
 * enqueues nothing (N = 20,000, M = 3, H = 91 needs 5 MiB; N = 80,000, M = 5,
 * H = 210 about 30 MiB).  The call allocates nothing and synchronises
 * nothing: the first call on a device looks up the array's address and the
 * device's shapes (host queries only).  Every call on a device shares that
 * device's array: calls that overlap in time on one device (different
 * streams, or different host threads) race and give undefined results;
 * calls on one stream are ordered and safe.  Levels beyond the 24th front are
 * peeled by one work-group (no cooperative launch), so inputs with very many
 * fronts are slower than with nsga3_select.
 */
#define NSGA3_NOALLOC_MAX_WORKSPACE (32u << 20)
nsga3_status nsga3_select_noalloc(const float *objs, int64_t N, int32_t M, const float *refs,
                                  int32_t H, int64_t K, int32_t *selected, int32_t *rank,
                                  int32_t *niche, float *dist, int32_t *dom_in, int32_t *dom_out,
                                  nsga3_info *info, hipStream_t stream);

/*
 * Batched selections: many independent problems (the islands or restarts of an
 * optimizer farm), each with its own N, M, H and K, run by one graph launch.
 * The fields of nsga3_problem mean what the arguments of nsga3_select mean;
 * every pointer is DEVICE memory owned by the caller.
 */
typedef struct {
    const float *objs;
    int64_t N;
    int32_t M;
    const float *refs;
    int32_t H;
    int64_t K;
    int32_t *selected;   /* required */
    int32_t *rank;       /* optional (NULL) */
    int32_t *niche;      /* optional */
    float *dist;         /* optional */
    int32_t *dom_in;     /* optional */
    int32_t *dom_out;    /* optional */
    nsga3_info *info;    /* optional */
} nsga3_problem;

typedef struct nsga3_plan nsga3_plan;

/*
 * Build a plan for B problems (probs: host array of B descriptors).  The plan
 * allocates one workspace per problem and captures, into one HIP graph, a
 * reset kernel and one persistent engine launch per distinct M (on parallel
 * graph branches).  An engine launch runs every problem of its M through all
 * stages of the selection as independent work items, so problems of very
 * different sizes and front counts share the GPU without per-problem
 * launches.  Synchronous; allocates.  The buffer pointers are baked into the
 * graph: the caller keeps them alive and may rewrite their contents between
 * launches.  Results of a launch are identical to running nsga3_select on
 * each problem; a problem whose data is bad (non-finite, bad reference row)
 * reports it in its own info and does not disturb the others.
 * Errors: NSGA3_E_INVALID for a bad descriptor (nothing is built),
 * NSGA3_E_NOMEM / NSGA3_E_HIP when allocation or capture fails.
 * When the context has profiling enabled (nsga3_profile) at creation, the
 * plan also collects the stage diagnostics of nsga3_plan_stage_times.
 */
nsga3_status nsga3_plan_create(nsga3_ctx *ctx, const nsga3_problem *probs, int32_t B,
                               nsga3_plan **out);

/* Launch the plan's graph on `stream` (asynchronous). */
nsga3_status nsga3_plan_launch(nsga3_plan *plan, hipStream_t stream);

/* Number of concurrent branches and of graph nodes (host query; either may be NULL). */
nsga3_status nsga3_plan_info(const nsga3_plan *plan, int32_t *branches, int64_t *nodes);

/* Free the plan (graph, workspaces).  The caller must make sure no launch of
 * the plan is still running.  NULL is ignored. */
void nsga3_plan_destroy(nsga3_plan *plan);

/* Work-item shapes the autotuner chose so far in this context, 5 int32 per
 * entry: M, N range (0: N < 2048, 1: < 8192, 2: < 32768, 3: larger), phase-A
 * items per level (pairwise decrements only), longest remaining list peeled in
 * one item (0: never), and largest front for that.  Writes at most `cap` entries to out (host) and the
 * number of entries to *count (host). */
nsga3_status nsga3_tuned_shapes(const nsga3_ctx *ctx, int32_t *out, int32_t cap, int32_t *count);

/* Keep the autotuner's choices across processes.  nsga3_tuned_save writes the
 * context's tuned shapes to the text file `path` (host path; written whole to
 * "<path>.tmp" and renamed): a header naming the device architecture and CU
 * count, then one line per (M, N range).  nsga3_tuned_load merges such a file
 * into the context (entries replace those of the same key), so plans created
 * afterwards with autotuning time only the groups still missing.  Errors:
 * NSGA3_E_INVALID for a missing, unreadable or malformed file (nothing is
 * loaded), NSGA3_E_UNSUPPORTED for a file tuned on another architecture or CU
 * count.  Host-only; neither touches the device. */
nsga3_status nsga3_tuned_save(const nsga3_ctx *ctx, const char *path);
nsga3_status nsga3_tuned_load(nsga3_ctx *ctx, const char *path);

/* Engine stages (index into the arrays of nsga3_plan_stage_times):
 *   0 keys and references, 1 radix histogram, 2 radix scatter, 3 sorted records,
 *   4 dominance counts, 5 split counts, 6 split writes, 7 peeling decrements,
 *   8 outputs in original order, 9 extreme points, 10 association,
 *   11 bucket scatter, 12 niche picks, 13 compaction counts, 14 compaction
 *   writes, 15 short-list split in one item, 16 remaining levels in one item,
 *   17 two-objective ranks in one ordered pass, 18 block tables of a front,
 *   19 done. */
#define NSGA3_PLAN_STAGES 20

/* Diagnostics of a plan created while profiling was enabled: per stage, the
 * block-milliseconds spent inside its work items and its epilogues, and the
 * number of items run; plus block-milliseconds spent finding work (probe) and
 * finding none (idle).  Sums over every worker block and every launch since
 * creation.  Synchronises the device.  Arrays are host double / int64_t
 * [NSGA3_PLAN_STAGES]; any pointer may be NULL.  NSGA3_E_UNSUPPORTED when the
 * plan collects no diagnostics. */
nsga3_status nsga3_plan_stage_times(const nsga3_plan *plan, double *item_ms,
                                    double *epilogue_ms, int64_t *items, double *probe_ms,
                                    double *idle_ms);

/* Phases of one nsga3_select call, for nsga3_phase_times. */
#define NSGA3_NUM_PHASES 6
/*   0  keys, ideal point, presort by key sum            (Alg. S.5 first step; sort prerequisite)
 *   1  dominance counts over all pairs                  (Listing 1, Eq. (6)-(7))
 *   2  front peeling and last front                     (Eq. (8)-(9), Alg. S.3)
 *   3  extreme points and intercepts                    (Alg. S.5)
 *   4  association and niche counts                     (Eq. (10)-(12))
 *   5  niche-preserving pick and output compaction      (Alg. S.1, Eq. (13)) */

/* Enable (1) or disable (0) phase timing.  While enabled, every nsga3_select
 * records NSGA3_NUM_PHASES + 1 HIP events on its stream (event creation may
 * allocate on the first calls).  Enabling clears the accumulated times. */
nsga3_status nsga3_profile(nsga3_ctx *ctx, int enable);

/* Synchronises on the recorded events and returns, per phase, the summed
 * duration in milliseconds over all calls since profiling was enabled
 * (ms: host double[NSGA3_NUM_PHASES]; calls: host, may be NULL), then clears. */
nsga3_status nsga3_phase_times(nsga3_ctx *ctx, double *ms, int64_t *calls);

/* Human-readable name of a status code (static string). */
const char *nsga3_status_string(nsga3_status s);

/* Library version as MAJOR*10000 + MINOR*100 + PATCH. */
int32_t nsga3_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NSGA3_H */
