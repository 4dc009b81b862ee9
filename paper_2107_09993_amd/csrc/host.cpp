// C ABI of the skyline library: argument checks (before any HIP call), grid
// choice, workspace layout and the launch sequence of the plain path.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/skycell.h"
#include "common.h"
#include "scan.h"
#include "host_internal.h"

namespace skycell {

static thread_local std::string g_last_error;

int set_error(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

int clear_error()
{
    g_last_error.clear();
    return SKYCELL_OK;
}

#define fail set_error
#define ok clear_error

// ---------------------------------------------------------------- grid choice
struct TuneEntry {
    int d;
    int log2n;
    int dtype;
    int g;
    int form;   // refine form for this grid: 0 lane, 1 wave, -1 not given
    int parts;  // wave form: waves per item, 0 not given
    int cls;    // input class (SKYCELL_CLASS_*) the row was tuned on, -1 any
};
static std::mutex g_tune_mu;
static std::vector<TuneEntry> g_tune;

// The table row for d and n among the rows `want` accepts, with the nearest
// log2 n no more than max_dist away: rows tuned on input class cls first (when
// cls >= 0), else rows for any class.  The caller holds g_tune_mu.
template <class Want>
static const TuneEntry *tune_row(int d, int64_t n, int cls, int max_dist, Want want)
{
    const int l2 = n > 1 ? (int)std::lround(std::log2((double)n)) : 0;
    for (int pass = cls >= 0 ? 0 : 1; pass < 2; ++pass) {
        const TuneEntry *best = nullptr;
        int best_dist = 1 << 30;
        for (const TuneEntry &e : g_tune) {
            if (e.d != d || !want(e)) continue;
            if (pass == 0 ? e.cls != cls : e.cls >= 0) continue;
            const int dist = std::abs(e.log2n - l2);
            if (dist < best_dist) {
                best_dist = dist;
                best = &e;
            }
        }
        if (best != nullptr && best_dist <= max_dist) return best;
    }
    return nullptr;
}

// Index bits per dimension for g columns: ceil(log2 g).
static int index_bits(int g)
{
    int r = 0;
    while ((1 << r) < g) ++r;
    return r;
}

// Size of the Morton index space, 2^(r*d), saturated above the cell budget.
uint64_t grid_cells(int g, int d)
{
    const int r = index_bits(g);
    if ((uint64_t)r * (uint64_t)d > 26) return (uint64_t)kMaxCells + 1;
    return (uint64_t)1 << (r * d);
}

static int default_grid(int64_t n, int d)
{
    // About two cells per point (one point per finest cell is the paper's
    // largest useful layer, Section VI), bounded below so tiny inputs still
    // get a grid and above by 2^24 cells.
    double target = 2.0 * (double)n;
    if (target < 4096.0) target = 4096.0;
    if (target > (double)(1u << 24)) target = (double)(1u << 24);
    int g = 1;
    while (grid_cells(g + 1, d) <= (uint64_t)target) ++g;
    return g;
}

// Batched instances: the tuning table entry for (d, n) under dtype code
// dtype + 2 (within the instance budget of 32 cells per point, at least 2^16
// and at most 2^24), else about two cells per point within 2^20 cells.
int choose_grid_batched(int64_t n, int d, int dtype)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const TuneEntry *e = tune_row(d, n, -1, 2, [&](const TuneEntry &t) { return t.dtype == dtype + 2; });
        const uint64_t cap = std::min<uint64_t>(1u << 24, std::max<uint64_t>(1u << 16, (uint64_t)n * 32u));
        if (e != nullptr && grid_cells(e->g, d) <= cap) return e->g;
    }
    double target = 2.0 * (double)n;
    if (target < 256.0) target = 256.0;
    if (target > (double)(1u << 20)) target = (double)(1u << 20);
    int g = 1;
    while (grid_cells(g + 1, d) <= (uint64_t)target) ++g;
    return g;
}

static int choose_grid(int64_t n, int d, int dtype, int cls = -1)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    // entries measured at sizes more than a factor ~2 away do not apply
    const TuneEntry *e = tune_row(d, n, cls, 1, [&](const TuneEntry &t) { return t.dtype == dtype; });
    if (e != nullptr && grid_cells(e->g, d) <= kMaxCells) return e->g;
    return default_grid(n, d);
}

// Whether the table holds rows tuned on one input class for single calls of
// this d, dtype and about this n (then the class of the input is worth
// computing before choosing the grid).
static bool has_class_rows(int64_t n, int d, int dtype)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const int l2 = n > 1 ? (int)std::lround(std::log2((double)n)) : 0;
    for (const TuneEntry &e : g_tune)
        if (e.d == d && e.dtype == dtype && e.cls >= 0 && std::abs(e.log2n - l2) <= 1) return true;
    return false;
}

// Query points per refine work item: the default for d, or SKYCELL_ITEMS_PER_LANE
// (1, 2 or 4) when set, for tuning sweeps.
static int items_per_lane(int d)
{
    static int env = -1;
    if (env < 0) {
        const char *v = getenv("SKYCELL_ITEMS_PER_LANE");
        const int e = v ? atoi(v) : 0;
        env = (e == 1 || e == 2 || e == 4) ? e : 0;
    }
    return env > 0 ? env : items_per_group(d);
}

// Refine form of a call: SKYCELL_REFINE_FORM=lane|wave (sweeps), else the
// tuning table's form for this (d, n, dtype) and grid, else the wave form when
// the grid is very coarse (at least 32 points per cell of the index space on
// average), where cells hold enough points to keep a wave busy.
static std::atomic<int> g_split_override{-1};  // slab split: -1 auto, 0 off, 1 on, 2 all that fit
static std::atomic<int> g_form_override{-2};  // -2 unread, -1 none, 0 lane, 1 wave, 2 tile, 3 plain lane

// The form the table (or the rule) gives, without the override.
static int table_form(int64_t n, int d, int g, int dtype, int cls)
{
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        const TuneEntry *e = tune_row(d, n, cls, 2, [&](const TuneEntry &t) {
            return t.g == g && t.form >= 0 && (t.dtype == dtype || t.dtype == dtype + 2);
        });
        if (e != nullptr) return e->form;
    }
    return (uint64_t)n >= 32ull * grid_cells(g, d) ? 1 : 0;
}

static int refine_form(int64_t n, int d, int g, int dtype, int cls)
{
    int ov = g_form_override.load();
    if (ov == -2) {
        const char *v = getenv("SKYCELL_REFINE_FORM");
        const int e = v == nullptr ? -1
                      : (strcmp(v, "wave") == 0   ? 1
                         : strcmp(v, "lane") == 0   ? 0
                         : strcmp(v, "tile") == 0   ? 2
                         : strcmp(v, "plain") == 0  ? 3
                                                    : -1);
        int expected = -2;
        g_form_override.compare_exchange_strong(expected, e);
        ov = g_form_override.load();
    }
    if (ov >= 0) return ov;
    return table_form(n, d, g, dtype, cls);
}

// Waves per item of the wave form: skycell_set_wave_parts / SKYCELL_WAVE_PARTS,
// else the tuning table's parts column for this (d, n, dtype) and grid, else 1.
// The candidates of a cone are dealt to the item's waves group by group, so the
// longest cones (cells near the top corner of a coarse grid, whose cone can
// hold most of the input) no longer run on one wave while the rest of the
// chip idles.
static std::atomic<int> g_parts_override{-2};  // -2 unread, 0 none, else the count

// Sampling gate of the pivot pre-filter (skycell_set_pivot_gate): 1 = on.
static std::atomic<int> g_pivot_gate{1};

// Cell prune of skycell_compute / skycell_compute_u16 (skycell_set_cell_prune).
static std::atomic<int> g_cell_prune{0};
int cell_prune_form() { return g_cell_prune.load(); }

// The waves per item the table gives, without the override.
static int table_parts(int64_t n, int d, int g, int dtype, int cls)
{
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const TuneEntry *e = tune_row(d, n, cls, 2, [&](const TuneEntry &t) {
        return t.g == g && t.form == 1 && t.parts >= 1 && (t.dtype == dtype || t.dtype == dtype + 2);
    });
    return e != nullptr ? e->parts : 1;
}

static int wave_parts(int64_t n, int d, int g, int dtype, int cls)
{
    int ov = g_parts_override.load();
    if (ov == -2) {
        const char *v = getenv("SKYCELL_WAVE_PARTS");
        int e = v ? atoi(v) : 0;
        if (e < 0 || e > kMaxWaveParts) e = 0;
        int expected = -2;
        g_parts_override.compare_exchange_strong(expected, e);
        ov = g_parts_override.load();
    }
    if (ov > 0) return ov;
    return table_parts(n, d, g, dtype, cls);
}

GridDesc pipeline_desc(int64_t n, int d, int g, int dtype, int cls)
{
    GridDesc gd = grid_desc(d, g);
    const int form = refine_form(n, d, g, dtype, cls);
    if (form == 2 && tile_form_supported(d, g)) {
        gd.tile = 1;
        return gd;
    }
    if (form == 3 || n >= kWrecMaxPoints) gd.plain = 1;
    if (form == 1) {
        gd.m = kWaveItemPoints;
        // items <= n, and items * parts work units must stay below 2^31
        const int64_t cap = std::max<int64_t>(1, ((int64_t)1 << 31) / std::max<int64_t>(n, 1) - 1);
        gd.parts = (int32_t)std::min<int64_t>(wave_parts(n, d, g, dtype, cls), cap);
    }
    return gd;
}

GridDesc grid_desc(int d, int g)
{
    GridDesc gd;
    memset(&gd, 0, sizeof(gd));
    gd.d = d;
    gd.g = g;
    gd.m = items_per_lane(d);
    gd.parts = 1;
    gd.r = index_bits(g);
    gd.cells = 1u << (gd.r * d);
    for (int k = 0; k < d; ++k)
        for (int b = 0; b < gd.r; ++b) gd.mask[k] |= 1u << (b * d + k);
    return gd;
}

// ---------------------------------------------------------------- workspace
static size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

size_t workspace_layout(int64_t n, int d, uint32_t cells, Workspace *ws, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) -> char * {
        char *p = base ? base + off : nullptr;
        off += align_up(bytes > 0 ? bytes : 1);
        return p;
    };
    const size_t nn = (size_t)n;
    Workspace w;
    w.cell_of = (uint32_t *)take(4 * nn);
    w.rank = (uint32_t *)take(4 * nn);
    w.cnt = (uint32_t *)take(4 * (size_t)cells);
    w.lc = (uint64_t *)take(8 * ((size_t)cells / 64 + 1));
    w.rec = (uint64_t *)take(8 * ((size_t)cells + 1));
    w.keys = (uint32_t *)take(4 * nn * (size_t)d);
    w.fkeys = (uint64_t *)take(8 * nn * (size_t)fine_words(d));
    w.sidx = (int32_t *)take(4 * nn);
    w.items = (uint2 *)take(8 * nn);
    w.flag = (uint8_t *)take(nn);
    const uint64_t tiles = std::max<uint64_t>(scan_tiles(cells), scan_tiles(nn));
    w.block_sums = (uint64_t *)take(8 * (size_t)(tiles + 1));
    w.ctr = (uint32_t *)take(4 * kCtrCount);
    w.survbits = (uint64_t *)take(8 * ((size_t)cells / 64 + 1));
    w.bcur = (uint32_t *)take(4 * (size_t)kMaxScatterBuckets * kNumXcd);
    w.stage = scatter_two_pass(n) ? (uint32_t *)take(4 * nn * (size_t)(((unsigned)d + 6u) & ~3u)) : nullptr;
    w.wrec = d <= kWrecMaxD ? (uint64_t *)take(16 * (size_t)cells) : nullptr;
    if (ws) *ws = w;
    return off;
}

// ---------------------------------------------------------------- devices
static std::mutex g_dev_mu;
static std::map<int, int> g_num_cus;

int device_cus(int dev)
{
    std::lock_guard<std::mutex> lk(g_dev_mu);
    auto it = g_num_cus.find(dev);
    if (it != g_num_cus.end()) return it->second;
    hipDeviceProp_t prop;
    int cus = 0;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) cus = prop.multiProcessorCount;
    if (cus < 1) cus = 1;
    g_num_cus[dev] = cus;
    return cus;
}

struct CachedWs {
    void *ptr = nullptr;
    size_t bytes = 0;
};
static std::mutex g_ws_mu;
static std::map<std::pair<int, hipStream_t>, CachedWs> g_ws_cache[kCacheCount];

int cached_buffer(int slot, int dev, hipStream_t st, size_t need, void **ptr)
{
    std::lock_guard<std::mutex> lk(g_ws_mu);
    CachedWs &c = g_ws_cache[slot][std::make_pair(dev, st)];
    if (c.bytes < need) {
        if (c.ptr != nullptr) {
            SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
            SKYCELL_HIP_CHECK(hipFree(c.ptr));
            c.ptr = nullptr;
            c.bytes = 0;
        }
        if (hipMalloc(&c.ptr, need) != hipSuccess) {
            c.ptr = nullptr;
            return fail(SKYCELL_E_NOMEM, "hipMalloc of %zu workspace bytes failed", need);
        }
        c.bytes = need;
    }
    *ptr = c.ptr;
    return SKYCELL_OK;
}

// ---------------------------------------------------------------- validation
int validate(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res,
                    int32_t value_bits, const int32_t *out_idx, const int32_t *out_count)
{
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return fail(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 0) return fail(SKYCELL_E_INVAL, "n = %lld is negative", (long long)n);
    if (n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld is not below 2^31", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D)
        return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (grid_res < 0) return fail(SKYCELL_E_INVAL, "grid_res = %d is negative", grid_res);
    if (out_count == nullptr) return fail(SKYCELL_E_INVAL, "out_count is NULL");
    if (n > 0 && points == nullptr) return fail(SKYCELL_E_INVAL, "points is NULL");
    if (n > 0 && out_idx == nullptr) return fail(SKYCELL_E_INVAL, "out_idx is NULL");
    if (dtype == SKYCELL_DTYPE_U16 && (value_bits < 1 || value_bits > 16))
        return fail(SKYCELL_E_RANGE, "value_bits = %d is outside [1, 16]", value_bits);
    return SKYCELL_OK;
}

int resolve_grid(int64_t n, int32_t d, int32_t dtype, int32_t grid_res, int *g_out, int cls)
{
    const int g = grid_res > 0 ? grid_res : choose_grid(n, d, dtype, cls);
    if (grid_cells(g, d) > kMaxCells)
        return fail(SKYCELL_E_RANGE,
                    "grid of %d columns in %d dimensions needs 2^(%d*%d) cells, over the budget of %u",
                    g, d, index_bits(g), d, (unsigned)kMaxCells);
    *g_out = g;
    return SKYCELL_OK;
}


// ---------------------------------------------------------------- phase timing
struct Profiler {
    bool on = false;
    int device = -1;
    hipEvent_t ev[SKYCELL_NUM_PHASES + 1] = {};
    bool recorded = false;
};
static thread_local Profiler g_prof;

static void prof_free()
{
    for (hipEvent_t &e : g_prof.ev)
        if (e != nullptr) {
            (void)hipEventDestroy(e);
            e = nullptr;
        }
    g_prof.recorded = false;
}

static int prof_mark(int i, hipStream_t st)
{
    if (!g_prof.on) return SKYCELL_OK;
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    if (g_prof.device != dev) {
        prof_free();
        g_prof.device = dev;
    }
    if (g_prof.ev[i] == nullptr) SKYCELL_HIP_CHECK(hipEventCreate(&g_prof.ev[i]));
    SKYCELL_HIP_CHECK(hipEventRecord(g_prof.ev[i], st));
    if (i == SKYCELL_NUM_PHASES) g_prof.recorded = true;
    return SKYCELL_OK;
}

#define SKYCELL_PROF(i)                             \
    do {                                            \
        int rc_ = prof_mark((i), st);               \
        if (rc_ != SKYCELL_OK) return rc_;          \
    } while (0)

int run_pipeline(const void *points, int32_t dtype, int64_t n, int32_t d, int g,
                 int32_t value_bits, int32_t *out_idx, int32_t *out_count, void *workspace,
                 uint64_t *stats, hipStream_t st, const PivotArgs *piv, const TreeScratch *tree, int cls)
{
    GridDesc gd = pipeline_desc(n, d, g, dtype, cls);
    // Slab split of the longest cone walks (cellops.h): measured on one MI355X,
    // anti-correlated n = 10^7, d = 8: 8.31 -> 8.16 ms per call; n = 10^6,
    // d = 8: -10%; but d = 6 (n = 10^7, uint16) +2% and n = 10^4 +4% (two more
    // launches), so it runs from d = 7 and 2^18 points.  The paper's tree prune
    // rewrites the cell records after the prefix-OR pass, so the split (sized
    // by that pass) stays off with it.
    const int split_mode = g_split_override.load();
    const bool split_auto = d >= 7 && n >= ((int64_t)1 << 18);
    if (tree == nullptr && lane_split(gd)) {
        if (split_mode == 2)
            gd.split = 2;
        else if (split_share() > 0u && (split_mode == 1 || (split_mode == -1 && split_auto)))
            gd.split = 1;
    }
    Workspace ws;
    workspace_layout(n, d, gd.cells, &ws, (char *)workspace);
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    const int cus = device_cus(dev);
    SKYCELL_PROF(0);
    SKYCELL_HIP_CHECK(launch_init(ws, gd, stats, st));
    SKYCELL_HIP_CHECK(launch_quantize_hist(points, dtype, n, gd, value_bits, ws, st));
    SKYCELL_PROF(1);
    SKYCELL_HIP_CHECK(launch_cell_prune(gd, ws, n, stats, st));
    if (tree != nullptr) {
        const int rho = gd.r;
        SKYCELL_HIP_CHECK(run_shrink_tree(ws.cnt, d, rho, *tree, nullptr, nullptr, st));
        SKYCELL_HIP_CHECK(apply_shrink_tree(*tree, rho, ws, gd.cells, stats, st));
    }
    const bool pivots = piv != nullptr && piv->k > 0;
    if (pivots) {
        SKYCELL_HIP_CHECK(launch_pivot_gather((const float *)points, (uint32_t)n, d, piv->idx, piv->k, piv->ps,
                                              ws.ctr, st));
        SKYCELL_HIP_CHECK(launch_pivot_prune((const float *)points, (uint32_t)n, gd, ws, piv->ps, piv->k, stats,
                                             g_pivot_gate.load() != 0, st));
    }
    SKYCELL_PROF(2);
    SKYCELL_HIP_CHECK(launch_cell_scan(gd, ws, n, stats, st, pivots));
    SKYCELL_PROF(3);
    SKYCELL_HIP_CHECK(launch_scatter(points, dtype, n, gd, ws, value_bits, cus, st));
    SKYCELL_PROF(4);
    SKYCELL_HIP_CHECK(launch_refine(n, gd, ws, stats, cus, st));
    SKYCELL_PROF(5);
    SKYCELL_HIP_CHECK(launch_output(n, ws, out_idx, out_count, stats, st));
    SKYCELL_PROF(6);
    return ok();
}

// The paper's tree-form cell prune, when chosen (skycell_set_cell_prune) and the
// grid has g = 2^rho columns: its scratch, library-owned and kept per (device,
// stream).  *use is false when the prefix-OR prune applies.
static int tree_scratch_for(int d, int g, int dev, hipStream_t st, TreeScratch *ts, bool *use)
{
    *use = false;
    const GridDesc gd = grid_desc(d, g);
    if (cell_prune_form() != 1 || g < 2 || (g & (g - 1)) != 0 || (1 << gd.r) != g) return SKYCELL_OK;
    const size_t tneed = tree_scratch_layout(gd.cells, d, gd.r, nullptr, nullptr);
    void *tptr = nullptr;
    const int rc = cached_buffer(kCacheTree, dev, st, tneed, &tptr);
    if (rc != SKYCELL_OK) return rc;
    tree_scratch_layout(gd.cells, d, gd.r, ts, (char *)tptr);
    *use = true;
    return SKYCELL_OK;
}

// Input class of n points (SKYCELL_CLASS_*): a sample's moments on `st`, read
// back with one synchronisation of `st`.  -1 while `st` is being captured.
static int input_class_sync(const void *points, int32_t dtype, int64_t n, int32_t d, hipStream_t st, int *cls)
{
    *cls = -1;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    SKYCELL_HIP_CHECK(hipStreamIsCapturing(st, &cap));
    if (cap != hipStreamCaptureStatusNone) return SKYCELL_OK;
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    const size_t bytes = class_moments_bytes(d);
    void *dbuf = nullptr;
    int rc = cached_buffer(kCacheClass, dev, st, bytes, &dbuf);
    if (rc != SKYCELL_OK) return rc;
    static std::mutex mu;
    static double *host = nullptr;  // pinned, for the largest d, kept for the process
    std::lock_guard<std::mutex> lk(mu);
    if (host == nullptr) {
        void *h = nullptr;
        SKYCELL_HIP_CHECK(hipHostMalloc(&h, class_moments_bytes(SKYCELL_MAX_D), hipHostMallocDefault));
        host = (double *)h;
    }
    SKYCELL_HIP_CHECK(launch_class_moments(points, dtype, n, d, (double *)dbuf, st));
    SKYCELL_HIP_CHECK(hipMemcpyAsync(host, dbuf, bytes, hipMemcpyDeviceToHost, st));
    SKYCELL_HIP_CHECK(hipStreamSynchronize(st));
    *cls = class_from_moments(host, d, n);
    return SKYCELL_OK;
}

// Inputs below this size are not classified: the read-back would cost more
// than a differently tuned grid can save.
constexpr int64_t kClassMinPoints = 1 << 16;

static int compute_owned(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res,
                         int32_t value_bits, int32_t *out_idx, int32_t *out_count, void *stream)
{
    int rc = validate(points, dtype, n, d, grid_res, value_bits, out_idx, out_count);
    if (rc != SKYCELL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    int cls = -1;
    if (grid_res == 0 && n >= kClassMinPoints && has_class_rows(n, d, dtype) &&
        (rc = input_class_sync(points, dtype, n, d, st, &cls)) != SKYCELL_OK)
        return rc;
    int g = 0;
    if ((rc = resolve_grid(n, d, dtype, grid_res, &g, cls)) != SKYCELL_OK) return rc;
    if (n == 0) {
        SKYCELL_HIP_CHECK(launch_write_zero_count(out_count, st));
        return ok();
    }
    const size_t need = workspace_layout(n, d, grid_desc(d, g).cells, nullptr, nullptr);
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    void *ptr = nullptr;
    if ((rc = cached_buffer(kCacheWorkspace, dev, st, need, &ptr)) != SKYCELL_OK) return rc;
    TreeScratch ts;
    bool use_tree = false;
    if ((rc = tree_scratch_for(d, g, dev, st, &ts, &use_tree)) != SKYCELL_OK) return rc;
    return run_pipeline(points, dtype, n, d, g, value_bits, out_idx, out_count, ptr, nullptr, st, nullptr,
                        use_tree ? &ts : nullptr, cls);
}

}  // namespace skycell

using namespace skycell;

extern "C" {

int skycell_compute(const float *points, int64_t n, int32_t d, int32_t grid_res, int32_t *out_idx,
                    int32_t *out_count, void *stream)
{
    return compute_owned(points, SKYCELL_DTYPE_F32, n, d, grid_res, 16, out_idx, out_count, stream);
}

int skycell_compute_u16(const uint16_t *points, int64_t n, int32_t d, int32_t grid_res,
                        int32_t value_bits, int32_t *out_idx, int32_t *out_count, void *stream)
{
    return compute_owned(points, SKYCELL_DTYPE_U16, n, d, grid_res, value_bits, out_idx, out_count,
                         stream);
}

int skycell_workspace_bytes(int64_t n, int32_t d, int32_t grid_res, int32_t dtype, size_t *bytes)
{
    if (bytes == nullptr) return fail(SKYCELL_E_INVAL, "bytes is NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return fail(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (grid_res < 0) return fail(SKYCELL_E_INVAL, "grid_res = %d is negative", grid_res);
    int g = 0;
    int rc = resolve_grid(n, d, dtype, grid_res, &g);
    if (rc != SKYCELL_OK) return rc;
    *bytes = n == 0 ? 256 : workspace_layout(n, d, grid_desc(d, g).cells, nullptr, nullptr);
    return ok();
}

int skycell_compute_ws(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res,
                       int32_t value_bits, int32_t *out_idx, int32_t *out_count, void *workspace,
                       size_t ws_bytes, uint64_t *stats, void *stream)
{
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    int rc = validate(points, dtype, n, d, grid_res, value_bits, out_idx, out_count);
    if (rc != SKYCELL_OK) return rc;
    int g = 0;
    if ((rc = resolve_grid(n, d, dtype, grid_res, &g)) != SKYCELL_OK) return rc;
    hipStream_t st = (hipStream_t)stream;
    if (n == 0) {
        SKYCELL_HIP_CHECK(launch_write_zero_count(out_count, st));
        return ok();
    }
    const size_t need = workspace_layout(n, d, grid_desc(d, g).cells, nullptr, nullptr);
    if (workspace == nullptr || ws_bytes < need)
        return fail(SKYCELL_E_NOMEM, "workspace of %zu bytes is smaller than the %zu required",
                    workspace ? ws_bytes : (size_t)0, need);
    if (((uintptr_t)workspace & 255u) != 0) return fail(SKYCELL_E_INVAL, "workspace is not 256-byte aligned");
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    TreeScratch ts;
    bool use_tree = false;
    if ((rc = tree_scratch_for(d, g, dev, st, &ts, &use_tree)) != SKYCELL_OK) return rc;
    return run_pipeline(points, dtype, n, d, g, value_bits, out_idx, out_count, workspace, stats, st, nullptr,
                        use_tree ? &ts : nullptr);
}

int skycell_choose_grid(int64_t n, int32_t d, int32_t dtype, int32_t *grid_res)
{
    if (grid_res == nullptr) return fail(SKYCELL_E_INVAL, "grid_res is NULL");
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (n < 0) return fail(SKYCELL_E_INVAL, "n is negative");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return fail(SKYCELL_E_INVAL, "bad dtype %d", dtype);
    *grid_res = choose_grid(n, d, dtype);
    return ok();
}

int skycell_input_class(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t *cls, void *stream)
{
    if (points == nullptr || cls == nullptr) return fail(SKYCELL_E_INVAL, "points and cls must not be NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return fail(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 1 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    int c = -1;
    const int rc = input_class_sync(points, dtype, n, d, (hipStream_t)stream, &c);
    if (rc != SKYCELL_OK) return rc;
    if (c < 0) return fail(SKYCELL_E_INVAL, "the stream is being captured into a graph");
    *cls = c;
    return ok();
}

int skycell_choose_config(int64_t n, int32_t d, int32_t dtype, int32_t cls, int32_t *grid_res, int32_t *form,
                          int32_t *parts)
{
    if (grid_res == nullptr || form == nullptr || parts == nullptr)
        return fail(SKYCELL_E_INVAL, "grid_res, form and parts must not be NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return fail(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (cls < -1 || cls > SKYCELL_CLASS_ANTICORRELATED) return fail(SKYCELL_E_INVAL, "cls = %d is not -1, 0, 1 or 2", cls);
    const int g = choose_grid(n, d, dtype, cls);
    *grid_res = g;
    *form = table_form(n, d, g, dtype, cls);
    *parts = *form == 1 ? table_parts(n, d, g, dtype, cls) : 0;
    return ok();
}

int skycell_set_refine_form(int32_t form)
{
    if (form < -1 || form > 3) return fail(SKYCELL_E_INVAL, "form = %d is not -1, 0, 1, 2 or 3", form);
    g_form_override.store(form);
    return ok();
}

int skycell_set_slab_split(int32_t mode)
{
    if (mode < -1 || mode > 2) return fail(SKYCELL_E_INVAL, "mode = %d is not -1, 0, 1 or 2", mode);
    g_split_override.store(mode);
    return ok();
}

int skycell_set_pivot_gate(int32_t on)
{
    if (on != 0 && on != 1) return fail(SKYCELL_E_INVAL, "on = %d is not 0 or 1", on);
    g_pivot_gate.store(on);
    return ok();
}

int skycell_set_cell_prune(int32_t form)
{
    if (form != 0 && form != 1) return fail(SKYCELL_E_INVAL, "form = %d is not 0 or 1", form);
    g_cell_prune.store(form);
    return ok();
}

int skycell_set_wave_parts(int32_t parts)
{
    if (parts < 0 || parts > kMaxWaveParts)
        return fail(SKYCELL_E_INVAL, "parts = %d is outside [0, %d]", parts, kMaxWaveParts);
    g_parts_override.store(parts);
    return ok();
}

int skycell_load_tuning(const char *path)
{
    std::vector<TuneEntry> entries;
    if (path != nullptr) {
        FILE *f = fopen(path, "r");
        if (f == nullptr) return fail(SKYCELL_E_INVAL, "cannot open tuning table %s", path);
        char line[256];
        while (fgets(line, sizeof(line), f)) {
            if (line[0] == '#') continue;
            TuneEntry e;
            e.form = -1;
            e.parts = 0;
            e.cls = -1;
            const int got = sscanf(line, "%d %d %d %d %d %d %d", &e.d, &e.log2n, &e.dtype, &e.g, &e.form, &e.parts,
                                   &e.cls);
            if (got >= 4 && e.d >= 1 && e.d <= SKYCELL_MAX_D && e.g >= 1) {
                if (got < 5 || (e.form != 0 && e.form != 1)) e.form = -1;
                if (got < 6 || e.parts < 1 || e.parts > kMaxWaveParts) e.parts = 0;
                if (got < 7 || e.cls < 0 || e.cls > SKYCELL_CLASS_ANTICORRELATED) e.cls = -1;
                entries.push_back(e);
            }
        }
        fclose(f);
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune.swap(entries);
    return ok();
}

int skycell_workspace_layout(int64_t n, int32_t d, int32_t grid_res, int32_t dtype, size_t *offsets,
                             int32_t count)
{
    if (offsets == nullptr || count < 13) return fail(SKYCELL_E_INVAL, "offsets needs 13 entries");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16) return fail(SKYCELL_E_INVAL, "bad dtype %d", dtype);
    if (n < 0 || n >= ((int64_t)1 << 31)) return fail(SKYCELL_E_INVAL, "n = %lld out of range", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return fail(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (grid_res < 0) return fail(SKYCELL_E_INVAL, "grid_res = %d is negative", grid_res);
    int g = 0;
    int rc = resolve_grid(n, d, dtype, grid_res, &g);
    if (rc != SKYCELL_OK) return rc;
    Workspace w;
    char *const base = (char *)(uintptr_t)4096;  // any aligned base; offsets are relative
    const size_t total = workspace_layout(n, d, grid_desc(d, g).cells, &w, base);
    const void *ptrs[12] = {w.cell_of, w.rank, w.cnt, w.lc, w.rec, w.keys, w.fkeys, w.sidx, w.items,
                            w.flag, w.block_sums, w.ctr};
    for (int i = 0; i < 12; ++i) offsets[i] = (size_t)((const char *)ptrs[i] - base);
    offsets[12] = total;
    return ok();
}

int skycell_profile_enable(int32_t on)
{
    if (!on) prof_free();
    g_prof.on = on != 0;
    return ok();
}

int skycell_profile_read(float *ms, int32_t count)
{
    if (ms == nullptr || count < SKYCELL_NUM_PHASES) return fail(SKYCELL_E_INVAL, "ms needs %d entries", SKYCELL_NUM_PHASES);
    if (!g_prof.recorded) return fail(SKYCELL_E_INVAL, "no profiled call on this thread");
    SKYCELL_HIP_CHECK(hipEventSynchronize(g_prof.ev[SKYCELL_NUM_PHASES]));
    for (int i = 0; i < SKYCELL_NUM_PHASES; ++i) {
        float v = 0.f;
        SKYCELL_HIP_CHECK(hipEventElapsedTime(&v, g_prof.ev[i], g_prof.ev[i + 1]));
        ms[i] = v;
    }
    return ok();
}

const char *skycell_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
