// Batched selection engine (internal): many independent selections run by one
// persistent kernel per objective count.  Every instance advances through its
// own sequence of stages; a stage is a set of independent work items; the
// block that finishes the last item of a stage prepares the next one.  No
// block ever waits for another, so the launch needs no co-residency and can
// be captured in a graph.
#pragma once

#include "common.h"

namespace nsga3 {

constexpr int kEThreads = 256;
constexpr int kEChunk = 1024;      // points per item of the O(N) stages
constexpr int kERsTile = 2048;     // keys per radix-sort item
constexpr int kESplit = 512;       // list entries per split item
constexpr int kECmp = 2048;        // flags per compaction item
constexpr int kESmem = 12288;      // LDS dwords per worker block
// Presort key: the exact key sum (at most 36 bits for M <= 16, at most five
// 8-bit passes: the sort runs over key - min key, with as many passes as the
// instance's key range needs); for M = 2 the lexicographic pair (key_1, key_2)
// (eight passes), which is also a linear extension of dominance and lets the
// fronts be found in one ordered pass (kSRank2).
__host__ __device__ constexpr int radix_passes(int M) { return M == 2 ? 8 : 5; }

__host__ __device__ constexpr int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

enum EStage : int32_t {
    kSPrep = 0,   // order keys, key sums, ideal point, finiteness; unit references
    kSHist,       // radix histogram (arg = pass)
    kSScat,       // radix scatter (arg = pass)
    kSRecs,       // sorted records and run starts
    kSDom,        // dominance counts over the (i-chunk, j-tile) triangle
    kSSplitC,     // level split: per-item front / remaining counts (arg = level)
    kSSplitW,     // level split: ordered write of F_k and U_k
    kSPhaseA,     // F_k x U_k in-degree decrements (p0 = chunk, p1 = tiles)
    kSOrig,       // ranks and counts back to the original order
    kSExt,        // extreme-point and nadir partials
    kSAssoc,      // association, niche counts
    kSBScat,      // last-front members into reference buckets
    kSBRank,      // in-bucket ranks and picks
    kSCmpC,       // selection flags: per-item counts
    kSCmpW,       // selection flags: ordered write
    kSSplit1,     // level split of a short list in one item (arg = level)
    kSPeelTail,   // every remaining level in one item (arg = level already split)
    kSRank2,      // M = 2: every rank in one ordered pass (one item)
    kSBuildF,     // block tables of the front F_k (arg = level)
    kSDone,
};

// Lists up to this length split in one item (which also builds the front's
// tables): limits of 4096, 8192, 16384 and 32768 entries took 14.4, 13.9,
// 13.6 and 13.5 ms per launch on the mixed batch.
constexpr int kESplitOne = 64 * kESplit;
constexpr int kETailDefault = 2048;      // default EInst::tail_max
constexpr int kETailFrontDefault = 256;  // default EInst::tail_front

// Per-instance scalars (in the instance's workspace).
struct EScal {
    uint32_t err;
    uint32_t min_key[16];
    int32_t num_fronts, last_front, last_front_size, fallback;
    int64_t n_before, R;
    int32_t near_ties, level_V, ref_thr;
    uint32_t n_selected;
    int32_t rank2_overflow;  // the ordered pass found more fronts than it can hold
    int32_t rs_passes;       // radix passes the presort takes (from the key range)
    unsigned long long skey_min, skey_max;  // range of the presort keys (M >= 3)
    double z[16], a[16];
};

// Byte offsets of one instance's arrays inside its workspace.
struct ELayout {
    size_t skey0, skey1, sval0, sval1, hist, recs, runstart, runend, tabs, din, dout, rank_s;
    size_t fk0, fk1, uk0, uk1, urun0, urun1, ucnt0, ucnt1, spc, fsize, usize;
    size_t rank, niche, dist64, p_asf, p_idx, p_nad, rhat64, rhat32;
    size_t rho, bcount, bstart, bcursor, bd, bi, selflag, cmpc, scal, total;
};

__host__ __device__ inline ELayout elayout(int64_t N, int M, int H) {
    ELayout L;
    size_t c = 0;
    auto bump = [&c](size_t bytes) {
        const size_t o = c;
        c += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const size_t n = (size_t)N;
    const size_t MP = (size_t)rec_stride(M);
    const size_t nrs = (size_t)cdiv(N, kERsTile);
    const size_t nch = (size_t)cdiv(N, kEChunk);
    L.skey0 = bump(8 * n);
    L.skey1 = bump(8 * n);
    L.sval0 = bump(4 * n);
    L.sval1 = bump(4 * n);
    L.hist = bump(4 * 256 * nrs);
    L.recs = bump(4 * n * MP);
    L.runstart = bump(4 * n);
    L.runend = bump(4 * n);
    // 64-member tables (counts, peeling levels) or, for 4 <= M <= 10, the
    // larger 128-member tables of the counts
    const size_t tab_narrow = (size_t)cdiv(N, 64) * (size_t)blk_stride(M);
    const size_t tab_wide = (M >= 4 && M <= 10) ? (size_t)cdiv(N, 128) * (size_t)wide_blk_stride(M) : 0;
    L.tabs = bump(4 * (tab_narrow > tab_wide ? tab_narrow : tab_wide));
    L.din = bump(4 * n);
    L.dout = bump(4 * n);
    L.rank_s = bump(4 * n);
    L.fk0 = bump(4 * n * MP);
    L.fk1 = bump(4 * n * MP);
    L.uk0 = bump(4 * n * MP);
    L.uk1 = bump(4 * n * MP);
    L.urun0 = bump(4 * n);
    L.urun1 = bump(4 * n);
    L.ucnt0 = bump(4 * n);
    L.ucnt1 = bump(4 * n);
    L.spc = bump(4 * 2 * ((size_t)cdiv(N, kESplit) + 1));
    L.fsize = bump(4 * (n + 1));
    L.usize = bump(4 * (n + 1));
    L.rank = bump(4 * n);
    L.niche = bump(4 * n);
    L.dist64 = bump(8 * n);
    L.p_asf = bump(8 * nch * (size_t)M);
    L.p_idx = bump(4 * nch * (size_t)M);
    L.p_nad = bump(8 * nch * (size_t)M);
    L.rhat64 = bump(8 * (size_t)H * M);
    L.rhat32 = bump(4 * (size_t)H * M);
    L.rho = bump(4 * (size_t)H);
    L.bcount = bump(4 * (size_t)H);
    L.bstart = bump(4 * ((size_t)H + 1));
    L.bcursor = bump(4 * (size_t)H);
    L.bd = bump(8 * n);
    L.bi = bump(4 * n);
    L.selflag = bump(n);
    L.cmpc = bump(4 * ((size_t)cdiv(N, kECmp) + 1));
    L.scal = bump(sizeof(EScal));
    L.total = c;
    return L;
}

// One instance (host-written, read-only on the device).
struct EInst {
    const float *objs, *refs;
    int32_t *selected, *rank, *niche;
    float *dist;
    int32_t *dom_in, *dom_out;
    nsga3_info *info;
    char *ws;
    int64_t K;
    int32_t N, M, H;
    int32_t pa_items;   // pairwise phase-A items a level aims for (chunk size adapts)
    int32_t tail_max;   // remaining lists up to this length peel in one item (0: never) ...
    int32_t tail_front; // ... when the current front has at most this many points
    int32_t bit_peel;   // 1: front x remaining decrements by block bitsets (else pairwise)
    ELayout L;          // elayout(N, M, H)
};

// Per-instance progress word and stage parameters (one 64-byte line each).
struct alignas(64) EState {
    uint64_t word;      // [63:32] items claimed, [31:0] items in the stage
    uint32_t done;      // items finished
    int32_t stage, arg, n, p0, p1;
};

struct alignas(128) EGlobal {
    uint32_t finished;  // instances done
    uint32_t err;       // engine-level error bits (kErrBarrierTimeout: idle limit hit)
    uint32_t pad[30];
};

// Optional diagnostics, summed over blocks and launches (wall-clock ticks).
struct EStats {
    unsigned long long item[kSDone + 1];      // inside items, per stage
    unsigned long long epilogue[kSDone + 1];  // epilogues of completed stages
    unsigned long long items[kSDone + 1];     // items run, per stage
    unsigned long long probe;                 // successful searches for an item
    unsigned long long idle;                  // searches that found nothing
};

// Launches (engine.hip).  Instances [b0, b0 + nb) of `inst` must share M.
hipError_t engine_init(const EInst *inst, EState *st, EGlobal *g, int32_t B, int32_t nclass,
                       hipStream_t s);
// Runs instances [b0, b0 + nb) until each is done or reaches stop_stage
// (then parked with no items).
hipError_t engine_launch(int M, const EInst *inst, EState *st, int32_t b0, int32_t nb, EGlobal *g,
                         EStats *stats, int32_t stop_stage, int grid, hipStream_t s);
// Dominance counts of every parked instance as one ordinary launch; map[q]
// = (instance, item) of block q, nblocks blocks.
hipError_t engine_dom_launch(int M, const EInst *inst, const EState *st, const int2 *map,
                             int64_t nblocks, hipStream_t s);
// Moves parked instances [b0, b0 + nb) to the first peeling level; instances
// already done count as finished in g.
hipError_t engine_resume(const EInst *inst, EState *st, int32_t b0, int32_t nb, EGlobal *g,
                         hipStream_t s);
// Block-bitset dominance counts of every parked instance (bitdom.hip): block
// tables (bmap[q] = (instance, block), nb_build entries), then in-degrees and
// out-degrees (cmap[q] = (instance, work-group), nb_count entries).
// out_mode as LaunchCfg::out_mode; wide allows 128-member tables where the
// single-selection counts use them (engine_counts_wide).
hipError_t engine_bitdom_launch(int M, const EInst *inst, const EState *st, const int2 *bmap,
                                int64_t nb_build, const int2 *cmap, int64_t nb_count,
                                int out_mode, bool wide, hipStream_t s);
// Block tables and count work-groups of one instance for the launch above
// (same M, out_mode and wide).
void engine_bitdom_items(int64_t N, int M, int out_mode, bool wide, int64_t *n_build,
                         int64_t *n_count);
// Whether the launch above counts over 128-member tables.
bool engine_counts_wide(int M, int out_mode, bool wide);

// Number of dominance items of an instance of N points.
inline int64_t engine_dom_items(int64_t N) {
    const int64_t T = cdiv(N, 1024);
    return T * (T + 1) / 2;
}
int engine_blocks_per_cu(int M);

}  // namespace nsga3
