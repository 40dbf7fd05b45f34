// Host-side launchers for the libnsga3 kernels (internal interface).
#pragma once

#include "common.h"

namespace nsga3 {

// Phase-boundary hook (records a timing event when profiling is on).
struct Marker {
    void (*fn)(void *) = nullptr;
    void *arg = nullptr;
    void operator()() const {
        if (fn) fn(arg);
    }
};

// ---- sort_scan.hip --------------------------------------------------------
size_t radix_sort_temp_bytes(int64_t n);
void radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *k_alt, uint32_t *v_alt, int64_t n,
                      int nbits, uint32_t *temp, hipStream_t s, bool *in_alt);
size_t compact_temp_bytes(int64_t n);
// In-place exclusive scan of v[0..n) by one work-group; *total = the sum.
void scan_inplace(uint32_t *v, int64_t n, uint32_t *total, hipStream_t s);
// Writes at most `cap` indices; *total (device) receives the number of set flags.
void compact_flags(const uint8_t *flag, int64_t n, int32_t *out, int64_t cap, uint32_t *temp,
                   uint32_t *total, hipStream_t s);

// ---- dominance.hip --------------------------------------------------------
// Pointers into the workspace used by the sorting stage (a0-a3).
struct SortViews {
    const float *objs;
    int64_t N;
    int M;
    int64_t K;
    uint64_t *skey, *skey_alt;   // [N] key sums
    uint32_t *sval, *sval_alt;   // [N] point index (permutation)
    uint32_t *temp;              // radix-sort / scan scratch
    uint32_t *recs;              // [N * rec_stride(M)] sorted records
    int32_t *runstart;           // [N]
    int32_t *runend;             // [N] first position of the next key-sum run
    uint32_t *tabs_all;          // block tables over all sorted points
    uint32_t *tabs_lvl;          // block tables of the current front
    int32_t *dom_in_s, *dom_out_s, *rank_s;  // [N] in sorted order
    uint32_t *fk[2], *uk[2];     // peeling lists (records)
    int32_t *urun[2], *ucnt[2];  // peeling lists (run starts, remaining in-degree)
    int32_t *fsize;              // [N] front sizes per level
    int32_t *usize;              // [N] points still unranked after each level
    uint32_t *work;              // [kMaxHostLevels] phase-A work counters (zeroed per call)
    uint64_t *lbstate;           // [2 * lb_stride] split look-back state
    size_t lb_stride;
    uint32_t *blkcnt;            // [2 * max grid] per-block counts
    int32_t *rank, *dom_in, *dom_out;  // outputs in original order (dom_* may be null)
    int out_mode = -1;                 // as LaunchCfg::out_mode
    bool wide = true;                  // all-pairs counts with 128-member tables (M >= 4)
    bool wide_levels = false;          // peeling levels with 128-member front tables
    DevScalars *sc;
    GridBar *bar;                // grid-barrier state (zeroed per call)
    Marker mark;
};

constexpr int kMaxHostLevels = 64;

struct LaunchCfg {
    int num_cus;
    int peel_blocks_per_cu;     // cooperative tail kernel
    int phase_a_blocks_per_cu;  // per-level pairwise kernel
    int host_levels;            // peeling levels enqueued as ordinary launches
    bool bitsets;               // block-bitset pair kernels (else pairwise compares)
    bool tail_block;            // single-workgroup peeling tail (graph capture)
    int out_mode = -1;          // out-degrees: -1 by objective count, 0 from the in-degree
                                // pass, 1 by their own backward pass
    bool wide = true;           // 128-member tables for the all-pairs counts (M >= 4)
    bool wide_levels = false;   // 128-member front tables for the staged peeling levels
    // front sizes per level expected from the previous call (0: unknown);
    // they size launch grids only, every kernel covers any actual size
    int32_t fprev[kProfLevels] = {};
    // levels whose expected front has at most this many points build their
    // tables inside the level kernel (0: never)
    int32_t lds_build_max = 0;
};

// Points left before a peeling tail at or below which one work-group
// finishes the remaining levels (at most about 2e6 pair tests) instead of the
// cooperative grid.
constexpr int kTailOneBlockMax = 2048;

// Whether out-degrees come from the in-degree pass's probes (each dominating
// member counted in LDS) rather than a backward pass of their own.
bool fused_out_counts(int M, int out_mode);

hipError_t run_sort_stage(const SortViews &v, const LaunchCfg &cfg, hipStream_t s);

// ---- bitdom.hip -----------------------------------------------------------
hipError_t run_bit_counts(const SortViews &v, hipStream_t s);
// Block tables of all sorted points (tabs_all), as the count stage builds them.
hipError_t run_build_all_tables(const SortViews &v, hipStream_t s);
// Whether the count stage of v builds 128-member tables in tabs_all (which the
// 64-member probes of later stages cannot read).
bool counts_use_wide(const SortViews &v);
// tables_in_lds: no table-build launch; the level kernel builds the front's
// tables in LDS per item (for fronts expected to be small).
void run_bit_level(const SortViews &v, const uint32_t *fk, const uint32_t *uk, const int32_t *urun,
                   int32_t *ucnt, int level, unsigned grid, int32_t f_expect,
                   bool tables_in_lds, hipStream_t s);
size_t bit_tables_bytes(int64_t N, int M);    // all points: 64- or 128-member tables
size_t level_tables_bytes(int64_t N, int M);  // a front's 64-member tables

// ---- peel.hip -------------------------------------------------------------
hipError_t run_peel(const SortViews &v, const LaunchCfg &cfg, hipStream_t s);
// Largest cooperative grid the peeling tail may use for this M (0 on error).
int peel_max_blocks_per_cu(int M);
size_t split_state_entries(int64_t N);

// ---- variation.hip --------------------------------------------------------
hipError_t run_sbx_pm(const float *X, int64_t n, int d, const float *lower, const float *upper,
                      double eta_c, double eta_m, const float *r_sbx, const float *r_pm, float *out,
                      int32_t *status, hipStream_t s);
hipError_t run_gather(const float *X, int64_t N, int d, const int32_t *idx, int64_t K, float *out,
                      int32_t *status, hipStream_t s);

// ---- hype.hip -------------------------------------------------------------
// TensorHypE selection after the sort stage (ranks and the last front of n).
struct HypeViews {
    const float *objs;
    int64_t N;
    int M;
    int64_t n;                   // population size to keep
    const float *vref;           // [M] reference point (device)
    const float *U;              // [s * M] uniform draws (device)
    int64_t s;
    int32_t *selected;           // [n] ascending
    double *d;                   // [N] or null: HV estimate on rank <= l, -inf elsewhere
    const int32_t *rank;         // [N] original order (from the sort stage)
    const uint32_t *tabs_all;    // block tables of all points (sorted order)
    uint64_t *skey, *skey_alt;   // [N] sort keys (the presort's buffers, free by now)
    uint32_t *sval, *sval_alt;
    uint32_t *temp;              // radix-sort / scan scratch
    uint8_t *selflag;            // [N]
    DevScalars *sc;
    nsga3_info *info;
    void *extra;                 // hype_extra_bytes(N, M, s)
};
size_t hype_extra_bytes(int64_t N, int M, int64_t s);
hipError_t run_hype(const HypeViews &v, hipStream_t st);

// ---- rvea.hip -------------------------------------------------------------
// TensorRVEA angle-penalized distance selection (one elite per reference).
struct RveaViews {
    const float *objs;
    int64_t N;
    int M;
    const float *refs;
    int H;
    double penalty;              // M (t / t_max)^alpha, computed on the host
    int32_t *elite;              // [H]
    int32_t *assign;             // [N] or null (then in the workspace)
    double *apd;                 // [N] or null (then in the workspace)
    nsga3_info *info;            // or null
    void *ws;                    // rvea_workspace_bytes(N, M, H)
};
size_t rvea_workspace_bytes(int64_t N, int M, int H);
hipError_t run_rvea(const RveaViews &v, hipStream_t s);

// ---- select.hip -----------------------------------------------------------
size_t oneshot_temp_bytes(int64_t n);   // workspace temp needed by the one-shot niching
// nsga3_info from the call's device scalars (K selections expected).
void run_finalize(nsga3_info *info, int64_t K, const DevScalars *sc, hipStream_t s);
struct SelectViews {
    const float *objs;
    int64_t N;
    int M;
    const float *refs;
    int H;
    int64_t K;
    const int32_t *rank;         // [N] original order
    int32_t *niche;              // [N]
    float *dist;                 // [N] or null
    double *dist64;              // [N]
    double *rhat64;              // [H*M]
    float *rhat32;               // [H*M]
    uint16_t *rhat16;            // [Hpad*KP] bfloat16 (matrix-core screening)
    double *p_asf;               // [nb * M]
    int32_t *p_idx;              // [nb * M]
    double *p_nad;               // [nb * M]
    int32_t *rho, *bcount, *bstart, *bcursor;  // [H], [H], [H+1], [H]
    int32_t *gstart;             // [H+1] first rank work-group of each bucket
    double *bd;                  // [N] bucketed distances
    int32_t *bi;                 // [N] bucketed indices
    uint8_t *selflag;            // [N]
    uint32_t *temp;
    int32_t *selected;           // [K]
    nsga3_info *info;            // caller's, may be null
    DevScalars *sc;
    int assoc_mode;
    int niching_mode;            // NSGA3_NICHING_EXACT or NSGA3_NICHING_ONESHOT
    Marker mark;
};

int normalize_partial_blocks(int64_t N);
hipError_t run_refs(const float *refs, int H, int M, double *rhat64, float *rhat32,
                    uint16_t *rhat16, DevScalars *sc, hipStream_t s);
hipError_t run_select_stage(const SelectViews &v, hipStream_t s);
hipError_t run_init(DevScalars *sc, int32_t *zero_i32[], const int64_t zero_n[], int nzero,
                    hipStream_t s);

}  // namespace nsga3
