// C ABI of libnsga3: context, workspace and the environmental-selection entry
// point.  Host code only; the kernels live in dominance.hip, select.hip and
// sort_scan.hip.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <math.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <new>
#include <vector>

#include "engine.h"
#include "kernels.h"

using namespace nsga3;

struct nsga3_plan {
    int device = 0;
    int branches = 0;
    int64_t nodes = 0;
    bool engine = false;                 // batched engine (else a graph of single selections)
    void *ews = nullptr;                 // engine: every instance's workspace
    nsga3::EInst *d_inst = nullptr;      // engine: instance table (sorted by M)
    nsga3::EState *d_state = nullptr;
    nsga3::EGlobal *d_glob = nullptr;    // two per objective count (before / after the counts)
    int2 *d_map = nullptr;               // (instance, item) of every dominance-count block
    int2 *d_bmap = nullptr;              // (instance, block) of every block-table build
    int2 *d_cmap = nullptr;              // (instance, work-group) of the bitset count kernels
    bool bitdom = true;                  // block-bitset counts (else pairwise items)
    nsga3::EStats *d_stats = nullptr;    // engine diagnostics (plans created while profiling)
    int clock_khz = 0;
    std::vector<void *> ws;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

struct EngineShape {        // per-instance work-item shape of the batched engine
    int32_t pa_items;
    int32_t tail_max;
    int32_t tail_front;
};

struct nsga3_ctx {
    int device;
    char arch[64];                  // device architecture name (tuned-shape cache key)
    nsga3_options opt;
    std::map<std::pair<int, int>, EngineShape> tuned;  // (M, N range) -> fastest shape
    int num_cus;
    int peel_bpc[17];
    void *ws;
    size_t ws_bytes;
    bool profiling;
    int phase_a_bpc;
    bool bitsets;
    bool tail_block;
    int out_mode;                   // NSGA3_SEPARATE_OUT: LaunchCfg::out_mode
    int fixed_levels;               // > 0: always enqueue this many peeling levels
    double tail_work;               // peeling work left for the one-work-group tail
    int32_t lds_build_max;          // LaunchCfg::lds_build_max
    bool wide;                      // LaunchCfg::wide
    bool wide_levels;               // LaunchCfg::wide_levels
    bool engine_wide;               // batched counts over 128-member tables
    volatile int32_t *last_fronts;  // pinned: front count, then level sizes, of the latest call
    std::vector<hipEvent_t> ev_pool;   // NSGA3_NUM_PHASES + 1 events per recorded call
    size_t ev_used;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxPeelBlocksPerCu = 4;
constexpr int kDefaultHostLevels = 24;
constexpr int kPlanBranches = 8;   // concurrent graph branches of a batched plan
constexpr int kPlanLevels = 8;     // peeling levels enqueued per problem in a plan

struct Layout {
    size_t skey, skey_alt, sval, sval_alt, temp, recs, runstart, dom_in_s, dom_out_s, rank_s;
    size_t fk0, fk1, uk0, uk1, urun0, urun1, ucnt0, ucnt1, fsize, usize, work, lbstate, blkcnt;
    size_t runend, tabs_all, tabs_lvl;
    size_t lb_stride;
    size_t rank, niche, dist64, rhat64, rhat32, rhat16, p_asf, p_idx, p_nad;
    size_t rho, bcount, bstart, bcursor, gstart, bd, bi, selflag, sc, bar;
    size_t total;
};

size_t bump(size_t &cur, size_t bytes) {
    const size_t at = cur;
    cur += (bytes + kAlign - 1) / kAlign * kAlign;
    return at;
}

Layout layout_for(int64_t N, int M, int H, int max_grid) {
    Layout L;
    size_t c = 0;
    const size_t n = (size_t)N;
    const size_t MP = (size_t)rec_stride(M);
    size_t temp = radix_sort_temp_bytes(N);
    const size_t ct = compact_temp_bytes(N);
    if (ct > temp) temp = ct;
    const size_t ot = oneshot_temp_bytes(N);
    if (ot > temp) temp = ot;
    const int nparts = normalize_partial_blocks(N);
    L.skey = bump(c, 8 * n);
    L.skey_alt = bump(c, 8 * n);
    L.sval = bump(c, 4 * n);
    L.sval_alt = bump(c, 4 * n);
    L.temp = bump(c, temp);
    L.recs = bump(c, 4 * n * MP);
    L.runstart = bump(c, 4 * n);
    L.runend = bump(c, 4 * n);
    L.tabs_all = bump(c, bit_tables_bytes(N, M));
    L.tabs_lvl = bump(c, level_tables_bytes(N, M));
    L.dom_in_s = bump(c, 4 * n);
    L.dom_out_s = bump(c, 4 * n);
    L.rank_s = bump(c, 4 * n);
    L.fk0 = bump(c, 4 * n * MP);
    L.fk1 = bump(c, 4 * n * MP);
    L.uk0 = bump(c, 4 * n * MP);
    L.uk1 = bump(c, 4 * n * MP);
    L.urun0 = bump(c, 4 * n);
    L.urun1 = bump(c, 4 * n);
    L.ucnt0 = bump(c, 4 * n);
    L.ucnt1 = bump(c, 4 * n);
    L.fsize = bump(c, 4 * n);
    L.usize = bump(c, 4 * n);
    L.work = bump(c, 4 * (size_t)kMaxHostLevels);
    L.lb_stride = split_state_entries(N);
    L.lbstate = bump(c, 8 * 2 * L.lb_stride);
    L.blkcnt = bump(c, 8 * (size_t)max_grid);
    L.rank = bump(c, 4 * n);
    L.niche = bump(c, 4 * n);
    L.dist64 = bump(c, 8 * n);
    L.rhat64 = bump(c, 8 * (size_t)H * M);
    L.rhat32 = bump(c, 4 * (size_t)H * M);
    L.rhat16 = bump(c, 2 * (size_t)((H + 31) / 32 * 32) * (M <= 8 ? 8 : 16));
    L.p_asf = bump(c, 8 * (size_t)nparts * M);
    L.p_idx = bump(c, 4 * (size_t)nparts * M);
    L.p_nad = bump(c, 8 * (size_t)nparts * M);
    L.rho = bump(c, 4 * (size_t)H);
    L.bcount = bump(c, 4 * (size_t)H);
    L.bstart = bump(c, 4 * ((size_t)H + 1));
    L.bcursor = bump(c, 4 * (size_t)H);
    L.gstart = bump(c, 4 * ((size_t)H + 1));
    L.bd = bump(c, 8 * n);
    L.bi = bump(c, 4 * n);
    L.selflag = bump(c, n);
    L.sc = bump(c, sizeof(DevScalars));
    L.bar = bump(c, sizeof(GridBar));
    L.total = c;
    return L;
}

bool sizes_ok(int64_t N, int32_t M, int32_t H) {
    return N >= 1 && N <= 2147483647LL && M >= 2 && M <= 16 && H >= 1 && H <= 65535;
}

// Workspace sizes grow monotonically in N, M and H, so the layout for the
// largest request fits every smaller one.
const int kGridCap = 256 * 16;

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
            changed = hipSetDevice(dev) == hipSuccess;
        }
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

nsga3_status ensure_ws(nsga3_ctx *ctx, size_t need) {
    if (need <= ctx->ws_bytes) return NSGA3_OK;
    if (ctx->opt.max_workspace_bytes && need > ctx->opt.max_workspace_bytes) return NSGA3_E_NOMEM;
    if (getenv("NSGA3_TEST_FAIL_ALLOC")) return NSGA3_E_NOMEM;
    if (ctx->ws) {
        (void)hipFree(ctx->ws);
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    void *p = nullptr;
    if (hipMalloc(&p, need) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_NOMEM;
    }
    ctx->ws = p;
    ctx->ws_bytes = need;
    return NSGA3_OK;
}

// Phase boundary marker: records the next pooled event when profiling.
struct PhaseMarks {
    nsga3_ctx *ctx;
    hipStream_t s;
    bool on;
    PhaseMarks(nsga3_ctx *c, hipStream_t st) : ctx(c), s(st), on(c && c->profiling) {
        if (on && c->ev_used + NSGA3_NUM_PHASES + 1 > c->ev_pool.size()) {
            for (int q = 0; q <= NSGA3_NUM_PHASES; ++q) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) { on = false; return; }
                c->ev_pool.push_back(e);
            }
        }
    }
    void mark() {
        if (on) (void)hipEventRecord(ctx->ev_pool[ctx->ev_used++], s);
    }
};


// Peeling work (front size x points left, summed over the levels from the
// tail's first level on) at or below which the last levels go to one
// work-group instead of three launches each.  One work-group has a
// thousandth of the chip's lanes, so only nearly empty levels belong there
// (N = 200k, M = 5: peel 1.15 ms at 1e4 or 3e4, 1.21 at 1e5, 1.42 at 4e5).
constexpr double kTailPairWork = 1.0e4;
// Largest expected front (points) whose tables the level kernel builds in LDS
// per item instead of a table-build launch.
constexpr int32_t kLevelLdsBuildMax = 8192;

LaunchCfg ctx_cfg(const nsga3_ctx *ctx, int M, int64_t N) {
    LaunchCfg cfg;
    cfg.num_cus = ctx->num_cus;
    cfg.peel_blocks_per_cu = ctx->peel_bpc[M];
    cfg.phase_a_blocks_per_cu = ctx->phase_a_bpc;
    cfg.bitsets = ctx->bitsets;
    cfg.tail_block = ctx->tail_block;
    cfg.out_mode = ctx->out_mode;
    cfg.wide = ctx->wide;
    cfg.wide_levels = ctx->wide_levels;
    cfg.lds_build_max = ctx->lds_build_max;
    // The previous call's front count and level sizes arrive asynchronously
    // in pinned memory; they only size launches (a stale or torn read shifts
    // work between the enqueued levels and the tail, never the results).
    // Enqueue one level more than the previous call needed, or stop where the
    // work left is small enough for one work-group.
    const volatile int32_t *fb = ctx->last_fronts;
    const int prev = fb ? fb[0] : 0;
    int lv = prev > 0 ? prev + 1 : kDefaultHostLevels;
    if (prev > 0 && prev <= kProfLevels && fb[1 + prev - 1] == 0) {
        int32_t u[kProfLevels];
        bool ok = true;
        for (int k = 0; k < prev; ++k) {
            u[k] = fb[1 + k];
            const int64_t before = k ? u[k - 1] : N;
            if (u[k] < 0 || u[k] > before) ok = false;
        }
        if (ok) {
            for (int k = 0; k < prev; ++k) cfg.fprev[k] = (int32_t)((k ? u[k - 1] : N) - u[k]);
            double work = 0.0;
            int k0 = prev;
            for (int k = prev - 1; k >= 1; --k) {
                work += (double)cfg.fprev[k] * (double)u[k];
                if (work > ctx->tail_work || u[k - 1] > kTailOneBlockMax) break;
                k0 = k;
            }
            if (k0 < prev) lv = k0;
        }
    }
    if (ctx->fixed_levels > 0) lv = ctx->fixed_levels;
    if (lv > kMaxHostLevels) lv = kMaxHostLevels;
    if (lv < 1) lv = 1;
    cfg.host_levels = lv;
    return cfg;
}

struct EnqArgs {
    char *ws;
    LaunchCfg cfg;
    int assoc;
    int niching = NSGA3_NICHING_EXACT;
    nsga3_ctx *marks;                 // record phase events into this context, or null
    volatile int32_t *last_fronts;    // pinned slot for the front count and level sizes, or null
};

// Views of the sort stage (a0-a3) over the workspace w carved by L.
SortViews sort_views(char *w, const Layout &L, const nsga3_problem &p, int32_t *rank_o,
                     const Marker &mk, const LaunchCfg &cfg) {
#define WS(T, f) reinterpret_cast<T *>(w + L.f)
    const float *objs = p.objs;
    const int64_t N = p.N, K = p.K;
    const int32_t M = p.M;
    int32_t *dom_in = p.dom_in, *dom_out = p.dom_out;
    DevScalars *sc = WS(DevScalars, sc);
    SortViews sv;
    sv.objs = objs;
    sv.N = N;
    sv.M = M;
    sv.K = K;
    sv.skey = WS(uint64_t, skey);
    sv.skey_alt = WS(uint64_t, skey_alt);
    sv.sval = WS(uint32_t, sval);
    sv.sval_alt = WS(uint32_t, sval_alt);
    sv.temp = WS(uint32_t, temp);
    sv.recs = WS(uint32_t, recs);
    sv.runstart = WS(int32_t, runstart);
    sv.runend = WS(int32_t, runend);
    sv.tabs_all = WS(uint32_t, tabs_all);
    sv.tabs_lvl = WS(uint32_t, tabs_lvl);
    sv.dom_in_s = WS(int32_t, dom_in_s);
    sv.dom_out_s = WS(int32_t, dom_out_s);
    sv.rank_s = WS(int32_t, rank_s);
    sv.fk[0] = WS(uint32_t, fk0);
    sv.fk[1] = WS(uint32_t, fk1);
    sv.uk[0] = WS(uint32_t, uk0);
    sv.uk[1] = WS(uint32_t, uk1);
    sv.urun[0] = WS(int32_t, urun0);
    sv.urun[1] = WS(int32_t, urun1);
    sv.ucnt[0] = WS(int32_t, ucnt0);
    sv.ucnt[1] = WS(int32_t, ucnt1);
    sv.fsize = WS(int32_t, fsize);
    sv.usize = WS(int32_t, usize);
    sv.work = WS(uint32_t, work);
    sv.lbstate = WS(uint64_t, lbstate);
    sv.lb_stride = L.lb_stride;
    sv.blkcnt = WS(uint32_t, blkcnt);
    sv.rank = rank_o;
    sv.dom_in = dom_in;
    sv.dom_out = dom_out;
    sv.sc = sc;
    sv.bar = WS(GridBar, bar);
    sv.mark = mk;
    sv.wide = cfg.wide;
    sv.wide_levels = cfg.wide_levels;
    sv.out_mode = cfg.out_mode;
#undef WS
    return sv;
}

// Enqueues one whole selection on `stream` using the workspace at a.ws (sized
// by layout_for for the problem).  Allocates nothing; safe to capture.
hipError_t enqueue_select(const EnqArgs &a, const nsga3_problem &p, hipStream_t stream) {
    const float *objs = p.objs, *refs = p.refs;
    const int64_t N = p.N, K = p.K;
    const int32_t M = p.M, H = p.H;
    int32_t *selected = p.selected, *rank = p.rank, *niche = p.niche;
    float *dist = p.dist;
    nsga3_info *info = p.info;
    const Layout L = layout_for(N, M, H, kGridCap);
    char *w = a.ws;
#define WS(T, f) reinterpret_cast<T *>(w + L.f)
    DevScalars *sc = WS(DevScalars, sc);
    int32_t *rank_o = rank ? rank : WS(int32_t, rank);
    int32_t *niche_o = niche ? niche : WS(int32_t, niche);

    PhaseMarks marks(a.marks, stream);
    Marker mk;
    mk.fn = [](void *x) { static_cast<PhaseMarks *>(x)->mark(); };
    mk.arg = &marks;
    marks.mark();
    int32_t *zero_p[] = {WS(int32_t, dom_in_s), WS(int32_t, dom_out_s), WS(int32_t, rho),
                         WS(int32_t, bcount), WS(int32_t, bar), WS(int32_t, work),
                         WS(int32_t, lbstate)};
    const int64_t zero_n[] = {N, N, H, H, (int64_t)(sizeof(GridBar) / sizeof(int32_t)),
                              kMaxHostLevels, (int64_t)(2 * L.lb_stride)};
    hipError_t e = run_init(sc, zero_p, zero_n, 7, stream);
    if (e == hipSuccess)
        e = run_refs(refs, H, M, WS(double, rhat64), WS(float, rhat32), WS(uint16_t, rhat16), sc,
                     stream);

    SortViews sv = sort_views(w, L, p, rank_o, mk, a.cfg);
    const LaunchCfg &cfg = a.cfg;
    if (e == hipSuccess) e = run_sort_stage(sv, cfg, stream);
    if (e == hipSuccess && a.last_fronts)
        e = hipMemcpyAsync((void *)a.last_fronts, &sc->fb[0], sizeof(int32_t) * (1 + kProfLevels),
                           hipMemcpyDeviceToHost, stream);

    SelectViews xv;
    xv.objs = objs;
    xv.N = N;
    xv.M = M;
    xv.refs = refs;
    xv.H = H;
    xv.K = K;
    xv.rank = rank_o;
    xv.niche = niche_o;
    xv.dist = dist;
    xv.dist64 = WS(double, dist64);
    xv.rhat64 = WS(double, rhat64);
    xv.rhat32 = WS(float, rhat32);
    xv.rhat16 = WS(uint16_t, rhat16);
    xv.p_asf = WS(double, p_asf);
    xv.p_idx = WS(int32_t, p_idx);
    xv.p_nad = WS(double, p_nad);
    xv.rho = WS(int32_t, rho);
    xv.bcount = WS(int32_t, bcount);
    xv.bstart = WS(int32_t, bstart);
    xv.bcursor = WS(int32_t, bcursor);
    xv.gstart = WS(int32_t, gstart);
    xv.bd = WS(double, bd);
    xv.bi = WS(int32_t, bi);
    xv.selflag = WS(uint8_t, selflag);
    xv.temp = WS(uint32_t, temp);
    xv.selected = selected;
    xv.info = info;
    xv.sc = sc;
    xv.assoc_mode = a.assoc;
    xv.niching_mode = a.niching;
    xv.mark = mk;
#undef WS
    if (e == hipSuccess) e = run_select_stage(xv, stream);
    if (e != hipSuccess) (void)hipGetLastError();
    return e;
}

}  // namespace

// ---------------------------------------------------------------------------
// Allocation-free selection.  Its workspace is `scratch`, one array per device
// in the code object's own memory, so a call allocates nothing (for callers
// under graph capture or in loops that must not allocate).  In host code the
// array's name is only a stand-in: its device address is fetched once per
// device with hipGetSymbolAddress and kept in g_noalloc[device].
// ---------------------------------------------------------------------------
static __device__ __align__(256) char scratch[NSGA3_NOALLOC_MAX_WORKSPACE];

namespace {
constexpr int kNoallocMaxDevices = 64;
struct NoallocDevice {
    bool ready = false;
    nsga3_status status = NSGA3_OK;   // set-up result, kept for later calls
    char *scratch = nullptr;          // device address of `scratch` on this device
    int num_cus = 0;
    int peel_bpc[17] = {};
};
NoallocDevice g_noalloc[kNoallocMaxDevices];
std::mutex g_noalloc_mu;

// Once per device, with that device current: the array's address and the
// launch shapes (device queries only).
nsga3_status noalloc_setup(int dev, NoallocDevice **out) {
    std::lock_guard<std::mutex> lock(g_noalloc_mu);
    NoallocDevice &d = g_noalloc[dev];
    if (!d.ready) {
        d.ready = true;
        d.status = NSGA3_OK;
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) {
            (void)hipGetLastError();
            d.status = NSGA3_E_HIP;
        } else if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
            d.status = NSGA3_E_UNSUPPORTED;
        } else {
            void *ptr = nullptr;
            if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
                (void)hipGetLastError();
                d.status = NSGA3_E_HIP;
            } else {
                d.scratch = (char *)ptr;
                d.num_cus = prop.multiProcessorCount;
                for (int m = 2; m <= 16; ++m) {
                    const int nb = peel_max_blocks_per_cu(m);
                    d.peel_bpc[m] = nb < kMaxPeelBlocksPerCu ? nb : kMaxPeelBlocksPerCu;
                }
            }
        }
    }
    *out = &d;
    return d.status;
}
}  // namespace

extern "C" {

const char *nsga3_status_string(nsga3_status s) {
    // a C caller may pass any int: read the argument's bits, not the enum
    // value (a load outside the enumerators' range is undefined in C++)
    int v = 0;
    static_assert(sizeof(s) == sizeof(v), "status is int-sized");
    memcpy(&v, &s, sizeof(v));
    switch (v) {
        case NSGA3_OK: return "ok";
        case NSGA3_E_INVALID: return "invalid argument";
        case NSGA3_E_NONFINITE: return "non-finite objective or invalid reference direction";
        case NSGA3_E_NOMEM: return "out of device memory or over the workspace cap";
        case NSGA3_E_HIP: return "HIP runtime error";
        case NSGA3_E_UNSUPPORTED: return "unsupported device or launch mode";
    }
    return "unknown status";
}

int32_t nsga3_version(void) { return 100; }

nsga3_status nsga3_workspace_size(int64_t N, int32_t M, int32_t H, size_t *bytes) {
    if (!bytes || !sizes_ok(N, M, H)) return NSGA3_E_INVALID;
    *bytes = layout_for(N, M, H, kGridCap).total;
    return NSGA3_OK;
}

nsga3_status nsga3_create(nsga3_ctx **out, int device, const nsga3_options *opt) {
    if (!out) return NSGA3_E_INVALID;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) { (void)hipGetLastError(); return NSGA3_E_HIP; }
    if (device < 0 || device >= ndev) return NSGA3_E_INVALID;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return NSGA3_E_HIP;
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0) return NSGA3_E_UNSUPPORTED;
    int coop = 0;
    if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device) != hipSuccess || !coop)
        return NSGA3_E_UNSUPPORTED;
    nsga3_ctx *c = new (std::nothrow) nsga3_ctx();
    if (!c) return NSGA3_E_NOMEM;
    c->device = device;
    snprintf(c->arch, sizeof(c->arch), "%s", prop.gcnArchName);
    for (char *q = c->arch; *q; ++q)
        if (*q == ' ' || *q == '\n') *q = '_';
    c->opt.assoc = NSGA3_ASSOC_FP32;
    c->opt.autotune = 0;
    c->opt.max_workspace_bytes = 0;
    c->opt.niching = NSGA3_NICHING_EXACT;
    if (opt) c->opt = *opt;
    if ((c->opt.assoc != NSGA3_ASSOC_FP32 && c->opt.assoc != NSGA3_ASSOC_BF16) ||
        (c->opt.niching != NSGA3_NICHING_EXACT && c->opt.niching != NSGA3_NICHING_ONESHOT)) {
        delete c;
        return NSGA3_E_INVALID;
    }
    c->num_cus = prop.multiProcessorCount;
    DeviceGuard g(device);
    for (int m = 0; m <= 16; ++m) c->peel_bpc[m] = 0;
    // NSGA3_PEEL_BLOCKS_PER_CU overrides the co-resident blocks per CU of the
    // peeling kernel (tuning); it is clamped to what the device can co-schedule.
    int want = kMaxPeelBlocksPerCu;
    if (const char *e = getenv("NSGA3_PEEL_BLOCKS_PER_CU")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 16) want = v;
    }
    for (int m = 2; m <= 16; ++m) {
        int nb = peel_max_blocks_per_cu(m);
        c->peel_bpc[m] = nb < want ? nb : want;
        if (c->peel_bpc[m] < 1 || c->num_cus * c->peel_bpc[m] > kGridCap) {
            delete c;
            return NSGA3_E_UNSUPPORTED;
        }
    }
    c->ws = nullptr;
    c->ws_bytes = 0;
    c->profiling = false;
    c->ev_used = 0;
    c->fixed_levels = 0;
    // NSGA3_PAIRWISE=1 selects the pairwise-compare dominance kernels instead
    // of the block-bitset ones (same results; kept for comparison)
    c->bitsets = true;
    if (const char *e = getenv("NSGA3_PAIRWISE")) c->bitsets = atoi(e) == 0;
    // work-groups per CU of the per-level decrement kernels: the bitset level
    // kernel's 24 KiB chunks let six stay resident (peel at N = 200k, M = 5:
    // 1.090 ms with 6 per CU, 1.093 with 8, 1.111 with 4)
    c->phase_a_bpc = c->bitsets ? 6 : 8;
    // NSGA3_TAIL_BLOCK=1: finish peeling in one workgroup instead of the
    // cooperative grid (the form captured graphs use; same results)
    c->tail_block = false;
    if (const char *e = getenv("NSGA3_TAIL_BLOCK")) c->tail_block = atoi(e) != 0;
    // NSGA3_SEPARATE_OUT=1 / 0: out-degrees always by their own backward pass
    // / always from the in-degree pass's probes (same results); unset: chosen
    // by the objective count
    c->out_mode = -1;
    if (const char *e = getenv("NSGA3_SEPARATE_OUT")) c->out_mode = atoi(e) != 0 ? 1 : 0;
    // NSGA3_TAIL_WORK: pair tests (front size x points left, summed over the
    // last levels) at or below which those levels go to one work-group
    c->tail_work = kTailPairWork;
    if (const char *e = getenv("NSGA3_TAIL_WORK")) c->tail_work = atof(e);
    // NSGA3_WIDE_TABLES=0: all-pairs counts with 64-member tables for every M
    c->wide = !(getenv("NSGA3_WIDE_TABLES") && atoi(getenv("NSGA3_WIDE_TABLES")) == 0);
    // NSGA3_WIDE_LEVELS=1: 128-member front tables for the staged peeling
    // levels (4 <= M <= 10).  Off by default: at N = 200k, M = 5 the peel took
    // 1.30 ms against 1.09 (a wide table build per level, half the members per
    // item, five work-groups per CU instead of six).
    c->wide_levels = getenv("NSGA3_WIDE_LEVELS") && atoi(getenv("NSGA3_WIDE_LEVELS")) != 0;
    // NSGA3_ENGINE_WIDE=1: batched plans count over 128-member tables too
    // (4 <= M <= 10, unless NSGA3_WIDE_TABLES=0).  Off by default: beside the
    // other classes' engines the M = 5 counts of the 512-instance batch took
    // 2.83 ms against 2.68 (and the table builds 0.64 against 0.51).
    c->engine_wide = c->wide && getenv("NSGA3_ENGINE_WIDE") &&
                     atoi(getenv("NSGA3_ENGINE_WIDE")) != 0;
    // NSGA3_LEVEL_LDS_BUILD: largest expected front whose tables the level
    // kernel builds in LDS itself (0: always a table-build launch)
    c->lds_build_max = kLevelLdsBuildMax;
    if (const char *e = getenv("NSGA3_LEVEL_LDS_BUILD")) c->lds_build_max = atoi(e);
    if (const char *e = getenv("NSGA3_HOST_LEVELS")) {
        const int v = atoi(e);
        if (v >= 1 && v <= kMaxHostLevels) c->fixed_levels = v;
    }
    if (const char *e = getenv("NSGA3_PHASE_A_BLOCKS_PER_CU")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 32) c->phase_a_bpc = v;
    }
    c->last_fronts = nullptr;
    {
        void *h = nullptr;
        if (hipHostMalloc(&h, sizeof(int32_t) * (1 + kProfLevels), hipHostMallocDefault) == hipSuccess) {
            c->last_fronts = (volatile int32_t *)h;
            *c->last_fronts = 0;
        } else {
            (void)hipGetLastError();
        }
    }
    *out = c;
    return NSGA3_OK;
}

void nsga3_destroy(nsga3_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        if (ctx->ws) (void)hipFree(ctx->ws);
        if (ctx->last_fronts) (void)hipHostFree((void *)ctx->last_fronts);
        for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    }
    delete ctx;
}

nsga3_status nsga3_profile(nsga3_ctx *ctx, int enable) {
    if (!ctx) return NSGA3_E_INVALID;
    ctx->profiling = enable != 0;
    ctx->ev_used = 0;
    return NSGA3_OK;
}

nsga3_status nsga3_phase_times(nsga3_ctx *ctx, double *ms, int64_t *calls) {
    if (!ctx || !ms) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    for (int q = 0; q < NSGA3_NUM_PHASES; ++q) ms[q] = 0.0;
    const size_t per = NSGA3_NUM_PHASES + 1;
    const size_t n = ctx->ev_used / per;
    for (size_t c = 0; c < n; ++c) {
        hipEvent_t *e = &ctx->ev_pool[c * per];
        if (hipEventSynchronize(e[NSGA3_NUM_PHASES]) != hipSuccess) return NSGA3_E_HIP;
        for (int q = 0; q < NSGA3_NUM_PHASES; ++q) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, e[q], e[q + 1]) != hipSuccess) return NSGA3_E_HIP;
            ms[q] += (double)t;
        }
    }
    if (calls) *calls = (int64_t)n;
    ctx->ev_used = 0;
    return NSGA3_OK;
}

nsga3_status nsga3_reserve(nsga3_ctx *ctx, int64_t N_max, int32_t M_max, int32_t H_max) {
    if (!ctx || !sizes_ok(N_max, M_max, H_max)) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    return ensure_ws(ctx, layout_for(N_max, M_max, H_max, kGridCap).total);
}

nsga3_status nsga3_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                          const float *refs, int32_t H, int64_t K, int32_t *selected, int32_t *rank,
                          int32_t *niche, float *dist, int32_t *dom_in, int32_t *dom_out,
                          nsga3_info *info, hipStream_t stream) {
    if (!ctx || !objs || !refs || !selected) return NSGA3_E_INVALID;
    if (!sizes_ok(N, M, H) || K < 1 || K > N) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    const Layout L = layout_for(N, M, H, kGridCap);
    nsga3_status st = ensure_ws(ctx, L.total);
    if (st != NSGA3_OK) return st;
    EnqArgs a;
    a.ws = (char *)ctx->ws;
    a.cfg = ctx_cfg(ctx, M, N);
    a.assoc = (int)ctx->opt.assoc;
    a.niching = (int)ctx->opt.niching;
    a.marks = ctx->profiling ? ctx : nullptr;
    a.last_fronts = ctx->last_fronts;
    const nsga3_problem p = {objs, N, M, refs, H, K, selected, rank, niche, dist,
                             dom_in, dom_out, info};
    return enqueue_select(a, p, stream) == hipSuccess ? NSGA3_OK : NSGA3_E_HIP;
}

nsga3_status nsga3_select_noalloc(const float *objs, int64_t N, int32_t M, const float *refs,
                                  int32_t H, int64_t K, int32_t *selected, int32_t *rank,
                                  int32_t *niche, float *dist, int32_t *dom_in, int32_t *dom_out,
                                  nsga3_info *info, hipStream_t stream) {
    if (!objs || !refs || !selected) return NSGA3_E_INVALID;
    if (!sizes_ok(N, M, H) || K < 1 || K > N) return NSGA3_E_INVALID;
    const Layout L = layout_for(N, M, H, kGridCap);
    if (L.total > (size_t)NSGA3_NOALLOC_MAX_WORKSPACE) return NSGA3_E_NOMEM;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) { (void)hipGetLastError(); return NSGA3_E_HIP; }
    if (dev < 0 || dev >= kNoallocMaxDevices) return NSGA3_E_UNSUPPORTED;
    NoallocDevice *d = nullptr;
    const nsga3_status st = noalloc_setup(dev, &d);
    if (st != NSGA3_OK) return st;
    EnqArgs a;
    a.ws = d->scratch;
    a.cfg.num_cus = d->num_cus;
    a.cfg.peel_blocks_per_cu = d->peel_bpc[M];
    a.cfg.phase_a_blocks_per_cu = 6;
    a.cfg.host_levels = kDefaultHostLevels;
    a.cfg.bitsets = true;
    a.cfg.tail_block = true;          // no cooperative launch: capture-safe
    a.assoc = NSGA3_ASSOC_FP32;
    a.marks = nullptr;
    a.last_fronts = nullptr;
    const nsga3_problem p = {objs, N, M, refs, H, K, selected, rank, niche, dist,
                             dom_in, dom_out, info};
    return enqueue_select(a, p, stream) == hipSuccess ? NSGA3_OK : NSGA3_E_HIP;
}

nsga3_status nsga3_sbx_pm(const float *X, int64_t n, int32_t d, const float *lower,
                          const float *upper, double eta_c, double eta_m, const float *r_sbx,
                          const float *r_pm, float *offspring, int32_t *status, hipStream_t stream) {
    if (!X || !lower || !upper || !r_sbx || !r_pm || !offspring) return NSGA3_E_INVALID;
    if (n < 2 || n > 2147483647LL || d < 1 || !(eta_c >= 0.0) || !(eta_m >= 0.0) || !isfinite(eta_c) ||
        !isfinite(eta_m))
        return NSGA3_E_INVALID;
    if (run_sbx_pm(X, n, d, lower, upper, eta_c, eta_m, r_sbx, r_pm, offspring, status, stream) !=
        hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    return NSGA3_OK;
}

nsga3_status nsga3_gather_rows(const float *X, int64_t N, int32_t d, const int32_t *idx, int64_t K,
                               float *out, int32_t *status, hipStream_t stream) {
    if (!X || !idx || !out || N < 1 || N > 2147483647LL || d < 1 || K < 1) return NSGA3_E_INVALID;
    if (run_gather(X, N, d, idx, K, out, status, stream) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    return NSGA3_OK;
}

nsga3_status nsga3_hype_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                               const float *vref, const float *U, int64_t s, int64_t n,
                               int32_t *selected, double *d, int32_t *rank, nsga3_info *info,
                               hipStream_t stream) {
    if (!ctx || !objs || !vref || !U || !selected) return NSGA3_E_INVALID;
    if (!sizes_ok(N, M, 1) || n < 1 || n > N || s < 1 || s > 2147483647LL) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    const Layout L = layout_for(N, M, 1, kGridCap);
    const size_t extra = hype_extra_bytes(N, M, s);
    const nsga3_status st = ensure_ws(ctx, L.total + extra);
    if (st != NSGA3_OK) return st;
    char *w = (char *)ctx->ws;
#define WS(T, f) reinterpret_cast<T *>(w + L.f)
    DevScalars *sc = WS(DevScalars, sc);
    int32_t *rank_o = rank ? rank : WS(int32_t, rank);
    const LaunchCfg cfg = ctx_cfg(ctx, M, N);
    PhaseMarks marks(nullptr, stream);   // phase timing covers nsga3_select only
    Marker mk;
    mk.fn = [](void *x) { static_cast<PhaseMarks *>(x)->mark(); };
    mk.arg = &marks;
    int32_t *zero_p[] = {WS(int32_t, dom_in_s), WS(int32_t, dom_out_s), WS(int32_t, bar),
                         WS(int32_t, work), WS(int32_t, lbstate)};
    const int64_t zero_n[] = {N, N, (int64_t)(sizeof(GridBar) / sizeof(int32_t)), kMaxHostLevels,
                              (int64_t)(2 * L.lb_stride)};
    hipError_t e = run_init(sc, zero_p, zero_n, 5, stream);
    // ranks and the last front for a population of n (no out-degrees needed)
    const nsga3_problem p = {objs, N, M, vref, 1, n, selected, rank_o, nullptr, nullptr,
                             nullptr, nullptr, nullptr};
    SortViews sv = sort_views(w, L, p, rank_o, mk, cfg);
    if (e == hipSuccess) e = run_sort_stage(sv, cfg, stream);
    if (e == hipSuccess && ctx->last_fronts)
        e = hipMemcpyAsync((void *)ctx->last_fronts, &sc->fb[0], sizeof(int32_t) * (1 + kProfLevels),
                           hipMemcpyDeviceToHost, stream);
    // the sample probes read 64-member tables of all points
    if (e == hipSuccess && (!cfg.bitsets || counts_use_wide(sv))) e = run_build_all_tables(sv, stream);
    if (e == hipSuccess) {
        HypeViews hv;
        hv.objs = objs;
        hv.N = N;
        hv.M = M;
        hv.n = n;
        hv.vref = vref;
        hv.U = U;
        hv.s = s;
        hv.selected = selected;
        hv.d = d;
        hv.rank = rank_o;
        hv.tabs_all = WS(uint32_t, tabs_all);
        hv.skey = WS(uint64_t, skey);
        hv.skey_alt = WS(uint64_t, skey_alt);
        hv.sval = WS(uint32_t, sval);
        hv.sval_alt = WS(uint32_t, sval_alt);
        hv.temp = WS(uint32_t, temp);
        hv.selflag = WS(uint8_t, selflag);
        hv.sc = sc;
        hv.info = info;
        hv.extra = w + L.total;
        e = run_hype(hv, stream);
    }
#undef WS
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    return NSGA3_OK;
}

nsga3_status nsga3_rvea_select(nsga3_ctx *ctx, const float *objs, int64_t N, int32_t M,
                               const float *refs, int32_t H, int64_t t, int64_t t_max, double alpha,
                               int32_t *elite, int32_t *assign, double *apd, nsga3_info *info,
                               hipStream_t stream) {
    if (!ctx || !objs || !refs || !elite) return NSGA3_E_INVALID;
    if (N < 1 || N > 2147483647LL || M < 2 || M > 16 || H < 2 || H > 65535) return NSGA3_E_INVALID;
    if (t < 0 || t_max < 1 || !(alpha >= 0.0) || !isfinite(alpha)) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    const nsga3_status st = ensure_ws(ctx, rvea_workspace_bytes(N, M, H));
    if (st != NSGA3_OK) return st;
    RveaViews v;
    v.objs = objs;
    v.N = N;
    v.M = M;
    v.refs = refs;
    v.H = H;
    v.penalty = (double)M * pow((double)t / (double)t_max, alpha);
    v.elite = elite;
    v.assign = assign;
    v.apd = apd;
    v.info = info;
    v.ws = ctx->ws;
    if (run_rvea(v, stream) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    return NSGA3_OK;
}

static bool problem_ok(const nsga3_problem &p) {
    return p.objs && p.refs && p.selected && sizes_ok(p.N, p.M, p.H) && p.K >= 1 && p.K <= p.N;
}

static void plan_free(nsga3_plan *pl) {
    if (!pl) return;
    DeviceGuard g(pl->device);
    if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
    if (pl->graph) (void)hipGraphDestroy(pl->graph);
    for (hipEvent_t e : pl->events) (void)hipEventDestroy(e);
    for (hipStream_t st : pl->streams) (void)hipStreamDestroy(st);
    if (pl->cap) (void)hipStreamDestroy(pl->cap);
    for (void *w : pl->ws)
        if (w) (void)hipFree(w);
    if (pl->ews) (void)hipFree(pl->ews);
    if (pl->d_inst) (void)hipFree(pl->d_inst);
    if (pl->d_state) (void)hipFree(pl->d_state);
    if (pl->d_glob) (void)hipFree(pl->d_glob);
    if (pl->d_map) (void)hipFree(pl->d_map);
    if (pl->d_bmap) (void)hipFree(pl->d_bmap);
    if (pl->d_cmap) (void)hipFree(pl->d_cmap);
    if (pl->d_stats) (void)hipFree(pl->d_stats);
    delete pl;
}

// N ranges the tuner tells apart.
static int n_range(int64_t N) { return N < 2048 ? 0 : N < 8192 ? 1 : N < 32768 ? 2 : 3; }

static const EngineShape kShapeDefault = {8, nsga3::kETailDefault, nsga3::kETailFrontDefault};
static const EngineShape kShapeCandidates[] = {
    {8, 0, 0},        {8, 512, 128},     {8, 2048, 256},    {8, 8192, 256},
    {8, 8192, 1024},  {8, 32768, 256},   {8, 32768, 1024},  {32, 8192, 1024},
    {32, 0, 0},
};

constexpr int kTuneReps = 3;  // timed runs per candidate shape (median taken)

// Times the whole engine pipeline on one group of instances (all of one M),
// eagerly on `s`, for every candidate shape; returns the fastest.  The group's
// instances use their own workspaces; their outputs are overwritten (the plan
// launches overwrite them again).
static nsga3_status tune_group(nsga3_ctx *ctx, const std::vector<nsga3::EInst> &group, int grid,
                               hipStream_t s, EngineShape *best) {
    using namespace nsga3;
    const int32_t nb = (int32_t)group.size();
    std::vector<int2> map, cmap;  // block-table builds, count work-groups
    for (int32_t q = 0; q < nb; ++q) {
        int64_t nbld = 0, ncnt = 0;
        engine_bitdom_items(group[q].N, group[q].M, ctx->out_mode, ctx->engine_wide, &nbld,
                            &ncnt);
        for (int64_t t = 0; t < nbld; ++t) map.push_back(make_int2(q, (int)t));
        for (int64_t t = 0; t < ncnt; ++t) cmap.push_back(make_int2(q, (int)t));
    }
    const size_t nmap = map.size();
    map.insert(map.end(), cmap.begin(), cmap.end());
    EInst *d_inst = nullptr;
    EState *d_state = nullptr;
    EGlobal *d_glob = nullptr;
    int2 *d_map = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    nsga3_status st = NSGA3_OK;
    if (hipMalloc((void **)&d_inst, sizeof(EInst) * nb) != hipSuccess ||
        hipMalloc((void **)&d_state, sizeof(EState) * nb) != hipSuccess ||
        hipMalloc((void **)&d_glob, sizeof(EGlobal) * 2) != hipSuccess ||
        hipMalloc((void **)&d_map, sizeof(int2) * (map.empty() ? 1 : map.size())) != hipSuccess ||
        hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        (void)hipGetLastError();
        st = NSGA3_E_NOMEM;
    }
    if (st == NSGA3_OK && !map.empty() &&
        hipMemcpy(d_map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice) != hipSuccess)
        st = NSGA3_E_HIP;
    const int M = group[0].M;
    float best_ms = -1.0f;
    std::vector<EInst> cand(group);
    for (const EngineShape &sh : kShapeCandidates) {
        if (st != NSGA3_OK) break;
        // phase-A items per level only shape the pairwise decrements
        if (group[0].bit_peel && sh.pa_items != kShapeDefault.pa_items) continue;
        for (EInst &e : cand) {
            e.pa_items = sh.pa_items;
            e.tail_max = sh.tail_max;
            e.tail_front = sh.tail_front;
        }
        if (hipMemcpy(d_inst, cand.data(), sizeof(EInst) * nb, hipMemcpyHostToDevice) != hipSuccess) {
            st = NSGA3_E_HIP;
            break;
        }
        // one untimed run, then the median of kTuneReps timed runs
        float reps[kTuneReps];
        float ms = 0.0f;
        for (int rep = 0; rep <= kTuneReps && st == NSGA3_OK; ++rep) {
            hipError_t e = hipEventRecord(e0, s);
            if (e == hipSuccess) e = engine_init(d_inst, d_state, d_glob, nb, 2, s);
            if (e == hipSuccess) e = engine_launch(M, d_inst, d_state, 0, nb, d_glob, nullptr, kSDom, grid, s);
            if (e == hipSuccess)
                e = engine_bitdom_launch(M, d_inst, d_state, d_map, (int64_t)nmap, d_map + nmap,
                                         (int64_t)cmap.size(), ctx->out_mode, ctx->engine_wide, s);
            if (e == hipSuccess) e = engine_resume(d_inst, d_state, 0, nb, d_glob + 1, s);
            if (e == hipSuccess) e = engine_launch(M, d_inst, d_state, 0, nb, d_glob + 1, nullptr, kSDone, grid, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                (void)hipGetLastError();
                st = NSGA3_E_HIP;
            }
            if (rep > 0) reps[rep - 1] = ms;
        }
        if (st == NSGA3_OK) {
            std::sort(reps, reps + kTuneReps);
            ms = reps[kTuneReps / 2];
        }
        if (st == NSGA3_OK && (best_ms < 0.0f || ms < best_ms)) {
            best_ms = ms;
            *best = sh;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (d_inst) (void)hipFree(d_inst);
    if (d_state) (void)hipFree(d_state);
    if (d_glob) (void)hipFree(d_glob);
    if (d_map) (void)hipFree(d_map);
    return st;
}

// Batched plan through the engine: instances sorted by M, one persistent
// engine launch per objective count (on forked streams), all captured with
// the reset kernel into one graph.
static nsga3_status plan_create_engine(nsga3_ctx *ctx, const nsga3_problem *probs, int32_t B,
                                       nsga3_plan *pl) {
    using namespace nsga3;
    std::vector<int32_t> order(B);
    for (int32_t b = 0; b < B; ++b) order[b] = b;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t x, int32_t y) { return probs[x].M < probs[y].M; });
    std::vector<EInst> inst(B);
    std::vector<size_t> off(B);
    size_t total = 0;
    for (int32_t q = 0; q < B; ++q) {
        const nsga3_problem &p = probs[order[q]];
        off[q] = total;
        total += (elayout(p.N, p.M, p.H).total + 255) & ~(size_t)255;
    }
    if (ctx->opt.max_workspace_bytes && total > ctx->opt.max_workspace_bytes) return NSGA3_E_NOMEM;
    if (getenv("NSGA3_TEST_FAIL_ALLOC")) return NSGA3_E_NOMEM;
    if (hipMalloc(&pl->ews, total) != hipSuccess ||
        hipMalloc((void **)&pl->d_inst, sizeof(EInst) * (size_t)B) != hipSuccess ||
        hipMalloc((void **)&pl->d_state, sizeof(EState) * (size_t)B) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_NOMEM;
    }
    EngineShape base = kShapeDefault;
    if (const char *e = getenv("NSGA3_ENGINE_PA_ITEMS")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 1 << 20) base.pa_items = v;
    }
    if (const char *e = getenv("NSGA3_ENGINE_TAIL_MAX")) {
        const int v = atoi(e);
        if (v >= 0) base.tail_max = v;
    }
    if (const char *e = getenv("NSGA3_ENGINE_TAIL_FRONT")) {
        const int v = atoi(e);
        if (v >= 0) base.tail_front = v;
    }
    pl->bitdom = !(getenv("NSGA3_PAIRWISE") && atoi(getenv("NSGA3_PAIRWISE")) != 0);
    std::vector<std::pair<int32_t, int32_t>> cls;  // (first instance, count) per M
    for (int32_t q = 0; q < B; ++q) {
        const nsga3_problem &p = probs[order[q]];
        EInst &e = inst[q];
        e.objs = p.objs;
        e.refs = p.refs;
        e.selected = p.selected;
        e.rank = p.rank;
        e.niche = p.niche;
        e.dist = p.dist;
        e.dom_in = p.dom_in;
        e.dom_out = p.dom_out;
        e.info = p.info;
        e.ws = (char *)pl->ews + off[q];
        e.K = p.K;
        e.N = (int32_t)p.N;
        e.M = p.M;
        e.H = p.H;
        e.pa_items = base.pa_items;
        e.tail_max = base.tail_max;
        e.tail_front = base.tail_front;
        e.bit_peel = pl->bitdom ? 1 : 0;
        e.L = elayout(p.N, p.M, p.H);
        if (q == 0 || p.M != probs[order[q - 1]].M) cls.push_back({q, 0});
        cls.back().second++;
    }
    const int nclass = (int)cls.size();
    // dominance-count blocks of every class: (instance, item)
    std::vector<int2> map;
    std::vector<int64_t> map_off(nclass + 1, 0);
    for (int c = 0; c < nclass; ++c) {
        map_off[c] = (int64_t)map.size();
        for (int32_t q = cls[c].first; q < cls[c].first + cls[c].second; ++q) {
            const int64_t items = engine_dom_items(inst[q].N);
            for (int64_t t = 0; t < items; ++t) map.push_back(make_int2(q, (int)t));
        }
    }
    map_off[nclass] = (int64_t)map.size();
    // block-bitset form: table builds and count work-groups per class
    std::vector<int2> bmap, cmap;
    std::vector<int64_t> boff(nclass + 1, 0), coff(nclass + 1, 0);
    for (int c = 0; c < nclass; ++c) {
        boff[c] = (int64_t)bmap.size();
        coff[c] = (int64_t)cmap.size();
        for (int32_t q = cls[c].first; q < cls[c].first + cls[c].second; ++q) {
            int64_t nbld = 0, ncnt = 0;
            engine_bitdom_items(inst[q].N, inst[q].M, ctx->out_mode, ctx->engine_wide, &nbld,
                                &ncnt);
            for (int64_t t = 0; t < nbld; ++t) bmap.push_back(make_int2(q, (int)t));
            for (int64_t t = 0; t < ncnt; ++t) cmap.push_back(make_int2(q, (int)t));
        }
    }
    boff[nclass] = (int64_t)bmap.size();
    coff[nclass] = (int64_t)cmap.size();
    if (hipMalloc((void **)&pl->d_glob, sizeof(EGlobal) * (size_t)(2 * nclass)) != hipSuccess ||
        hipMalloc((void **)&pl->d_map, sizeof(int2) * (map.size() ? map.size() : 1)) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_NOMEM;
    }
    if (!map.empty() &&
        hipMemcpy(pl->d_map, map.data(), sizeof(int2) * map.size(), hipMemcpyHostToDevice) != hipSuccess)
        return NSGA3_E_HIP;
    if (hipMalloc((void **)&pl->d_bmap, sizeof(int2) * (bmap.size() ? bmap.size() : 1)) != hipSuccess ||
        hipMalloc((void **)&pl->d_cmap, sizeof(int2) * (cmap.size() ? cmap.size() : 1)) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_NOMEM;
    }
    if ((!bmap.empty() && hipMemcpy(pl->d_bmap, bmap.data(), sizeof(int2) * bmap.size(),
                                    hipMemcpyHostToDevice) != hipSuccess) ||
        (!cmap.empty() && hipMemcpy(pl->d_cmap, cmap.data(), sizeof(int2) * cmap.size(),
                                    hipMemcpyHostToDevice) != hipSuccess))
        return NSGA3_E_HIP;
    if (ctx->opt.autotune) {
        // shapes per (M, N range): tune the groups the context has not seen
        std::map<std::pair<int, int>, std::vector<int32_t>> groups;
        for (int32_t q = 0; q < B; ++q) groups[{inst[q].M, n_range(inst[q].N)}].push_back(q);
        hipStream_t ts = nullptr;
        if (hipStreamCreateWithFlags(&ts, hipStreamNonBlocking) != hipSuccess) return NSGA3_E_HIP;
        nsga3_status st = NSGA3_OK;
        for (auto &kv : groups) {
            if (ctx->tuned.count(kv.first)) continue;
            std::vector<EInst> g;
            for (int32_t q : kv.second) g.push_back(inst[q]);
            EngineShape best = kShapeDefault;
            st = tune_group(ctx, g, ctx->num_cus, ts, &best);
            if (st != NSGA3_OK) break;
            ctx->tuned[kv.first] = best;
        }
        (void)hipStreamDestroy(ts);
        if (st != NSGA3_OK) return st;
        for (int32_t q = 0; q < B; ++q) {
            const EngineShape &sh = ctx->tuned[{inst[q].M, n_range(inst[q].N)}];
            inst[q].pa_items = sh.pa_items;
            inst[q].tail_max = sh.tail_max;
            inst[q].tail_front = sh.tail_front;
        }
    }
    if (hipMemcpy(pl->d_inst, inst.data(), sizeof(EInst) * (size_t)B, hipMemcpyHostToDevice) !=
        hipSuccess)
        return NSGA3_E_HIP;
    if (ctx->profiling) {
        if (hipMalloc((void **)&pl->d_stats, sizeof(EStats)) != hipSuccess ||
            hipMemset(pl->d_stats, 0, sizeof(EStats)) != hipSuccess ||
            hipDeviceGetAttribute(&pl->clock_khz, hipDeviceAttributeWallClockRate, ctx->device) !=
                hipSuccess) {
            (void)hipGetLastError();
            return NSGA3_E_NOMEM;
        }
    }
    hipError_t e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
    for (int c = 0; c < nclass && e == hipSuccess; ++c) {
        hipStream_t bs;
        e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
        if (e == hipSuccess) pl->streams.push_back(bs);
    }
    // events: one per class for each of the two engine phases, fork, join,
    // one per class for its counts
    for (int c = 0; c < 3 * nclass + 2 && e == hipSuccess; ++c) {
        hipEvent_t ev;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) pl->events.push_back(ev);
    }
    if (e != hipSuccess) return NSGA3_E_HIP;
    pl->branches = nclass;
    std::vector<int> grid(nclass);
    for (int c = 0; c < nclass; ++c) {
        // one resident worker per CU and class: idle workers that poll for
        // items slow the working ones down more than extra workers help
        const int M = inst[cls[c].first].M;
        const int occ = engine_blocks_per_cu(M);
        int bpc = 1;
        if (const char *ev = getenv("NSGA3_ENGINE_BLOCKS_PER_CU")) {
            const int v = atoi(ev);
            if (v >= 1 && v <= occ) bpc = v;
        }
        grid[c] = ctx->num_cus * bpc;
    }
    hipEvent_t *ev = pl->events.data();
    auto counts = [&](int c, hipStream_t st) {
        const int M = inst[cls[c].first].M;
        if (pl->bitdom)
            return engine_bitdom_launch(M, pl->d_inst, pl->d_state, pl->d_bmap + boff[c],
                                        boff[c + 1] - boff[c], pl->d_cmap + coff[c],
                                        coff[c + 1] - coff[c], ctx->out_mode, ctx->engine_wide, st);
        return engine_dom_launch(M, pl->d_inst, pl->d_state, pl->d_map + map_off[c],
                                 map_off[c + 1] - map_off[c], st);
    };
    // Each class runs its three phases on its own branch, so one class's counts
    // overlap other classes' engines (6 % shorter launches on the mixed batch
    // than counts with no engine running, which NSGA3_PLAN_OVERLAP=0 selects).
    // The counts of the classes with M >= 3 run one class at a time, ascending
    // M, which starts the longest peeling first; the two-objective classes'
    // counts start as soon as their own phase 1 ends (mode 2), before any
    // phase-3 engine holds the CUs: behind the chain they ran starved beside
    // two engines (4.9 ms instead of 0.3).  512-instance batch: 11.1-11.2 ms
    // per launch against 11.5-11.7 with them chained last (mode 1); all
    // counts together (mode 0) 11.4 ms; mode 3 chains the M >= 3 classes in
    // descending M instead (11.7 ms).  NSGA3_PLAN_COUNT_ORDER selects.
    const bool overlap = !(getenv("NSGA3_PLAN_OVERLAP") && atoi(getenv("NSGA3_PLAN_OVERLAP")) == 0);
    int order_mode = 2;
    if (const char *oe = getenv("NSGA3_PLAN_COUNT_ORDER")) order_mode = atoi(oe);
    const bool ordered = order_mode != 0;
    // mode 2: the two-objective classes' counts start right after their own
    // phase 1, beside the other classes' chain instead of after it
    const bool m2_free = order_mode >= 2;
    std::vector<int> corder(nclass);
    for (int c = 0; c < nclass; ++c) corder[c] = c;
    const bool descending = order_mode == 3;  // mode 3: as 2, M >= 3 classes in descending M
    std::stable_sort(corder.begin(), corder.end(), [&](int x, int y) {
        const int mx = inst[cls[x].first].M, my = inst[cls[y].first].M;
        return std::make_pair(mx == 2, descending ? -mx : mx) <
               std::make_pair(my == 2, descending ? -my : my);
    });
    hipEvent_t *cev = ev + 2 * nclass + 2;  // counts of class c done
    // phase 1 (branch per class): keys, presort, records; parked before the counts
    e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = engine_init(pl->d_inst, pl->d_state, pl->d_glob, B, 2 * nclass, pl->cap);
    if (e == hipSuccess) e = hipEventRecord(ev[2 * nclass], pl->cap);
    for (int c = 0; c < nclass && e == hipSuccess; ++c) {
        const int M = inst[cls[c].first].M;
        hipStream_t bs = pl->streams[c];
        e = hipStreamWaitEvent(bs, ev[2 * nclass], 0);
        if (e == hipSuccess)
            e = engine_launch(M, pl->d_inst, pl->d_state, cls[c].first, cls[c].second, pl->d_glob + c,
                              pl->d_stats, kSDom, grid[c], bs);
    }
    // (in count order, so that each wait names an event already recorded)
    for (int q = 0; q < nclass && e == hipSuccess; ++q) {
        const int c = corder[q];
        const int M = inst[cls[c].first].M;
        hipStream_t bs = pl->streams[c];
        if (overlap) {
            if (ordered && q > 0 && !(m2_free && M == 2))
                e = hipStreamWaitEvent(bs, cev[corder[q - 1]], 0);
            if (e == hipSuccess) e = counts(c, bs);
            if (ordered && e == hipSuccess) e = hipEventRecord(cev[c], bs);
            if (e == hipSuccess)
                e = engine_resume(pl->d_inst, pl->d_state, cls[c].first, cls[c].second,
                                  pl->d_glob + nclass + c, bs);
            if (e == hipSuccess)
                e = engine_launch(M, pl->d_inst, pl->d_state, cls[c].first, cls[c].second,
                                  pl->d_glob + nclass + c, pl->d_stats, kSDone, grid[c], bs);
        }
        if (e == hipSuccess) e = hipEventRecord(ev[c], bs);
        if (e == hipSuccess) e = hipStreamWaitEvent(pl->cap, ev[c], 0);
    }
    if (!overlap) {
        // phase 2: the dominance counts of every instance, with no engine
        // running (the engines' cache invalidations would keep these
        // launches' data cold)
        for (int c = 0; c < nclass && e == hipSuccess; ++c) e = counts(c, pl->cap);
        if (e == hipSuccess) e = hipEventRecord(ev[2 * nclass + 1], pl->cap);
        // phase 3 (branch per class): peeling, normalisation, association, niching, output
        for (int c = 0; c < nclass && e == hipSuccess; ++c) {
            const int M = inst[cls[c].first].M;
            hipStream_t bs = pl->streams[c];
            e = hipStreamWaitEvent(bs, ev[2 * nclass + 1], 0);
            if (e == hipSuccess)
                e = engine_resume(pl->d_inst, pl->d_state, cls[c].first, cls[c].second,
                                  pl->d_glob + nclass + c, bs);
            if (e == hipSuccess)
                e = engine_launch(M, pl->d_inst, pl->d_state, cls[c].first, cls[c].second,
                                  pl->d_glob + nclass + c, pl->d_stats, kSDone, grid[c], bs);
            if (e == hipSuccess) e = hipEventRecord(ev[nclass + c], bs);
            if (e == hipSuccess) e = hipStreamWaitEvent(pl->cap, ev[nclass + c], 0);
        }
    }
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(pl->cap, &graph);
    if (e == hipSuccess) e = e2;
    pl->graph = graph;
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e == hipSuccess) {
        size_t nn = 0;
        if (hipGraphGetNodes(pl->graph, nullptr, &nn) == hipSuccess) pl->nodes = (int64_t)nn;
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    pl->engine = true;
    return NSGA3_OK;
}

nsga3_status nsga3_plan_create(nsga3_ctx *ctx, const nsga3_problem *probs, int32_t B,
                               nsga3_plan **out) {
    if (!ctx || !probs || !out || B < 1) return NSGA3_E_INVALID;
    *out = nullptr;
    for (int32_t b = 0; b < B; ++b)
        if (!problem_ok(probs[b])) return NSGA3_E_INVALID;
    DeviceGuard g(ctx->device);
    nsga3_plan *pl = new (std::nothrow) nsga3_plan();
    if (!pl) return NSGA3_E_NOMEM;
    pl->device = ctx->device;
    const char *mode = getenv("NSGA3_PLAN_MODE");
    // the engine implements the exact niching only: one-shot plans are graphs
    // of single selections
    if (!(mode && strcmp(mode, "graph") == 0) && ctx->opt.niching == NSGA3_NICHING_EXACT) {
        const nsga3_status st = plan_create_engine(ctx, probs, B, pl);
        if (st != NSGA3_OK) {
            plan_free(pl);
            return st;
        }
        *out = pl;
        return NSGA3_OK;
    }
    int nbr = kPlanBranches;
    if (const char *e = getenv("NSGA3_PLAN_BRANCHES")) {
        const int v = atoi(e);
        if (v >= 1 && v <= 64) nbr = v;
    }
    if (nbr > B) nbr = B;
    pl->branches = nbr;
    int levels = kPlanLevels;
    if (const char *e = getenv("NSGA3_PLAN_LEVELS")) {
        const int v = atoi(e);
        if (v >= 1 && v <= kMaxHostLevels) levels = v;
    }
    // balance the branches: largest problems first, each to the least loaded branch
    std::vector<int32_t> order(B);
    for (int32_t b = 0; b < B; ++b) order[b] = b;
    auto cost = [&](int32_t b) { return (double)probs[b].N * (double)probs[b].N * probs[b].M; };
    std::sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return cost(x) > cost(y); });
    std::vector<std::vector<int32_t>> members(nbr);
    std::vector<double> load(nbr, 0.0);
    std::vector<size_t> need(nbr, 0);
    for (int32_t b : order) {
        int best = 0;
        for (int q = 1; q < nbr; ++q)
            if (load[q] < load[best]) best = q;
        members[best].push_back(b);
        load[best] += cost(b);
        const size_t n = layout_for(probs[b].N, probs[b].M, probs[b].H, kGridCap).total;
        if (n > need[best]) need[best] = n;
    }
    for (int q = 0; q < nbr; ++q) std::sort(members[q].begin(), members[q].end());
    nsga3_status st = NSGA3_OK;
    hipError_t e = hipSuccess;
    pl->ws.assign(nbr, nullptr);
    for (int q = 0; q < nbr && st == NSGA3_OK; ++q) {
        if (ctx->opt.max_workspace_bytes && need[q] > ctx->opt.max_workspace_bytes) st = NSGA3_E_NOMEM;
        else if (hipMalloc(&pl->ws[q], need[q]) != hipSuccess) { (void)hipGetLastError(); st = NSGA3_E_NOMEM; }
    }
    if (st == NSGA3_OK) {
        e = hipStreamCreateWithFlags(&pl->cap, hipStreamNonBlocking);
        for (int q = 0; q < nbr && e == hipSuccess; ++q) {
            hipStream_t bs;
            e = hipStreamCreateWithFlags(&bs, hipStreamNonBlocking);
            if (e == hipSuccess) pl->streams.push_back(bs);
        }
        for (int q = 0; q <= nbr && e == hipSuccess; ++q) {
            hipEvent_t ev;
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
            if (e == hipSuccess) pl->events.push_back(ev);
        }
        if (e != hipSuccess) st = NSGA3_E_HIP;
    }
    if (st == NSGA3_OK) {
        e = hipStreamBeginCapture(pl->cap, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) e = hipEventRecord(pl->events[nbr], pl->cap);
        for (int q = 0; q < nbr && e == hipSuccess; ++q) {
            e = hipStreamWaitEvent(pl->streams[q], pl->events[nbr], 0);
            for (int32_t b : members[q]) {
                if (e != hipSuccess) break;
                EnqArgs a;
                a.ws = (char *)pl->ws[q];
                a.cfg = ctx_cfg(ctx, probs[b].M, probs[b].N);
                a.cfg.tail_block = true;       // cooperative launches cannot be captured
                a.cfg.host_levels = levels;
                for (int k = 0; k < kProfLevels; ++k) a.cfg.fprev[k] = 0;  // replays see other data
                a.assoc = (int)ctx->opt.assoc;
                a.niching = (int)ctx->opt.niching;
                a.marks = nullptr;
                a.last_fronts = nullptr;
                e = enqueue_select(a, probs[b], pl->streams[q]);
            }
            if (e == hipSuccess) e = hipEventRecord(pl->events[q], pl->streams[q]);
            if (e == hipSuccess) e = hipStreamWaitEvent(pl->cap, pl->events[q], 0);
        }
        hipGraph_t graph = nullptr;
        const hipError_t e2 = hipStreamEndCapture(pl->cap, &graph);
        if (e == hipSuccess) e = e2;
        pl->graph = graph;
        if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
        if (e == hipSuccess) {
            size_t nn = 0;
            if (hipGraphGetNodes(pl->graph, nullptr, &nn) == hipSuccess) pl->nodes = (int64_t)nn;
        }
        if (e != hipSuccess) { (void)hipGetLastError(); st = NSGA3_E_HIP; }
    }
    if (st != NSGA3_OK) {
        plan_free(pl);
        return st;
    }
    *out = pl;
    return NSGA3_OK;
}

nsga3_status nsga3_plan_launch(nsga3_plan *plan, hipStream_t stream) {
    if (!plan || !plan->exec) return NSGA3_E_INVALID;
    DeviceGuard g(plan->device);
    if (hipGraphLaunch(plan->exec, stream) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    return NSGA3_OK;
}

nsga3_status nsga3_plan_info(const nsga3_plan *plan, int32_t *branches, int64_t *nodes) {
    if (!plan) return NSGA3_E_INVALID;
    if (branches) *branches = plan->branches;
    if (nodes) *nodes = plan->nodes;
    return NSGA3_OK;
}

nsga3_status nsga3_tuned_shapes(const nsga3_ctx *ctx, int32_t *out, int32_t cap, int32_t *count) {
    if (!ctx || !count || cap < 0 || (cap > 0 && !out)) return NSGA3_E_INVALID;
    int32_t n = 0;
    for (const auto &kv : ctx->tuned) {
        if (n < cap) {
            int32_t *r = out + 5 * n;
            r[0] = kv.first.first;
            r[1] = kv.first.second;
            r[2] = kv.second.pa_items;
            r[3] = kv.second.tail_max;
            r[4] = kv.second.tail_front;
        }
        ++n;
    }
    *count = n;
    return NSGA3_OK;
}

// Tuned-shape cache file: a header line "nsga3-tuned-shapes 1 <arch> <CUs>",
// then one line "M n_range pa_items tail_max tail_front" per entry.
nsga3_status nsga3_tuned_save(const nsga3_ctx *ctx, const char *path) {
    if (!ctx || !path || !*path) return NSGA3_E_INVALID;
    char tmp[4096];
    if (snprintf(tmp, sizeof(tmp), "%s.tmp", path) >= (int)sizeof(tmp)) return NSGA3_E_INVALID;
    FILE *f = fopen(tmp, "w");
    if (!f) return NSGA3_E_INVALID;
    bool ok = fprintf(f, "nsga3-tuned-shapes 1 %s %d\n", ctx->arch, ctx->num_cus) > 0;
    for (const auto &kv : ctx->tuned)
        ok = ok && fprintf(f, "%d %d %d %d %d\n", kv.first.first, kv.first.second,
                           kv.second.pa_items, kv.second.tail_max, kv.second.tail_front) > 0;
    ok = (fclose(f) == 0) && ok;
    if (!ok || rename(tmp, path) != 0) {
        (void)remove(tmp);
        return NSGA3_E_INVALID;
    }
    return NSGA3_OK;
}

nsga3_status nsga3_tuned_load(nsga3_ctx *ctx, const char *path) {
    if (!ctx || !path) return NSGA3_E_INVALID;
    FILE *f = fopen(path, "r");
    if (!f) return NSGA3_E_INVALID;
    char magic[32] = {0}, arch[64] = {0};
    int version = 0, cus = 0;
    nsga3_status st = NSGA3_OK;
    if (fscanf(f, "%31s %d %63s %d", magic, &version, arch, &cus) != 4 ||
        strcmp(magic, "nsga3-tuned-shapes") != 0 || version != 1) {
        st = NSGA3_E_INVALID;
    } else if (strcmp(arch, ctx->arch) != 0 || cus != ctx->num_cus) {
        st = NSGA3_E_UNSUPPORTED;  // tuned on another device
    }
    std::vector<std::pair<std::pair<int, int>, EngineShape>> rows;
    while (st == NSGA3_OK) {
        int m = 0, r = 0, pa = 0, tm = 0, tf = 0;
        const int got = fscanf(f, "%d %d %d %d %d", &m, &r, &pa, &tm, &tf);
        if (got == EOF) break;
        if (got != 5 || m < 2 || m > 16 || r < 0 || r > 3 || pa < 1 || pa > (1 << 20) || tm < 0 ||
            tf < 0) {
            st = NSGA3_E_INVALID;
            break;
        }
        rows.push_back({{m, r}, EngineShape{pa, tm, tf}});
    }
    fclose(f);
    if (st != NSGA3_OK) return st;  // nothing is taken from a rejected file
    for (const auto &row : rows) ctx->tuned[row.first] = row.second;
    return NSGA3_OK;
}

static_assert(nsga3::kSDone + 1 == NSGA3_PLAN_STAGES, "stage list and header disagree");

nsga3_status nsga3_plan_stage_times(const nsga3_plan *plan, double *item_ms, double *epilogue_ms,
                                    int64_t *items, double *probe_ms, double *idle_ms) {
    if (!plan) return NSGA3_E_INVALID;
    if (!plan->d_stats || plan->clock_khz <= 0) return NSGA3_E_UNSUPPORTED;
    DeviceGuard g(plan->device);
    nsga3::EStats h;
    if (hipDeviceSynchronize() != hipSuccess ||
        hipMemcpy(&h, plan->d_stats, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) {
        (void)hipGetLastError();
        return NSGA3_E_HIP;
    }
    const double per_ms = (double)plan->clock_khz;  // ticks per millisecond
    for (int q = 0; q < NSGA3_PLAN_STAGES; ++q) {
        if (item_ms) item_ms[q] = (double)h.item[q] / per_ms;
        if (epilogue_ms) epilogue_ms[q] = (double)h.epilogue[q] / per_ms;
        if (items) items[q] = (int64_t)h.items[q];
    }
    if (probe_ms) *probe_ms = (double)h.probe / per_ms;
    if (idle_ms) *idle_ms = (double)h.idle / per_ms;
    return NSGA3_OK;
}

void nsga3_plan_destroy(nsga3_plan *plan) { plan_free(plan); }

}  // extern "C"
