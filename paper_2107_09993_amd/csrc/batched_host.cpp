// C ABI of the batched path.  A plan lays out every instance's workspace in
// one allocation and, at the first run (and again when a run passes other
// buffers), captures the single-instance path of every instance into one
// hipGraph: the instances are spread round-robin over kBranches fork-joined
// capture streams, largest estimated work first, so the graph holds that many
// independent chains the runtime may overlap.  A run is one hipGraphLaunch.
// Every node is a kernel of the single-instance path (no memset nodes: the
// path clears its counters with a kernel).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <numeric>
#include <vector>

#include "../../include/skycell.h"
#include "common.h"
#include "host_internal.h"

using namespace skycell;

namespace {

constexpr int kMaxBranches = 64;

// Fork-joined capture streams: independent chains of instances that the graph
// may run side by side.  Small instances leave most of the chip idle, so the
// throughput grows with the number of chains up to about 24-32 (4096 mixed
// instances: 8 chains 650, 16 chains 1104, 32 chains 1122 instances/s).
// SKYCELL_BATCH_BRANCHES overrides the default of 32 (1..kMaxBranches).
static int batch_branches()
{
    static int b = -1;
    if (b < 0) {
        const char *v = getenv("SKYCELL_BATCH_BRANCHES");
        const int e = v ? atoi(v) : 0;
        b = (e >= 1 && e <= kMaxBranches) ? e : 32;
    }
    return b;
}

// Cell budget of one batched instance: 32 cells per point, at least 2^16 and at
// most 2^24, so that the plan's workspace stays proportional to its points.
uint64_t batch_max_cells(int64_t n)
{
    const uint64_t c = (uint64_t)n * 32u;
    return c < (1u << 16) ? (1u << 16) : (c > (1u << 24) ? (1u << 24) : c);
}

}  // namespace

struct skycell_plan {
    int device = 0;
    int dtype = SKYCELL_DTYPE_F32;
    int value_bits = 16;
    int32_t num_inst = 0;
    std::vector<int64_t> n;
    std::vector<int32_t> d;
    std::vector<int32_t> g;
    std::vector<uint32_t> order;   // capture order: largest estimated work first
    std::vector<int64_t> pts_off;  // [num_inst + 1] element offsets
    std::vector<int64_t> out_off;  // [num_inst + 1]
    std::vector<size_t> ws_off;    // [num_inst + 1] byte offsets in the workspace
    char *d_ws = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t launched = nullptr;  // recorded after every launch of exec
    bool launched_pending = false;
    const void *bound_points = nullptr;
    int32_t *bound_out_idx = nullptr;
    int32_t *bound_out_count = nullptr;
};

namespace {

// Destroys the captured graph once its last launch has finished (a run that
// passes other buffers recaptures while the previous launch may still run).
void drop_graph(skycell_plan *p)
{
    if (p->launched_pending && p->launched) (void)hipEventSynchronize(p->launched);
    p->launched_pending = false;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->bound_points = nullptr;
    p->bound_out_idx = nullptr;
    p->bound_out_count = nullptr;
}

void plan_free(skycell_plan *p)
{
    if (p == nullptr) return;
    drop_graph(p);
    if (p->launched) (void)hipEventDestroy(p->launched);
    if (p->d_ws) (void)hipFree(p->d_ws);
    delete p;
}

// Capture streams and fork/join events, created once per device and kept for
// the life of the process (creating and destroying tens of streams and events
// at every capture is costly and was the heaviest churn of the plan lifecycle).
struct CaptureKit {
    bool ready = false;
    hipStream_t origin = nullptr;
    hipStream_t branch[kMaxBranches] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kMaxBranches] = {};
};
constexpr int kMaxKitDevices = 64;
static std::mutex g_kit_mu;
static CaptureKit g_kit[kMaxKitDevices];

static hipError_t capture_kit(int dev, CaptureKit **out)
{
    if (dev < 0 || dev >= kMaxKitDevices) return hipErrorInvalidDevice;
    CaptureKit &k = g_kit[dev];
    if (!k.ready) {
        hipError_t e = hipStreamCreateWithFlags(&k.origin, hipStreamNonBlocking);
        for (int i = 0; i < kMaxBranches && e == hipSuccess; ++i)
            e = hipStreamCreateWithFlags(&k.branch[i], hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&k.fork, hipEventDisableTiming);
        for (int i = 0; i < kMaxBranches && e == hipSuccess; ++i)
            e = hipEventCreateWithFlags(&k.join[i], hipEventDisableTiming);
        if (e != hipSuccess) return e;  // what was created is kept for the next attempt
        k.ready = true;
    }
    *out = &k;
    return hipSuccess;
}

// Capture every instance's path with this run's buffers into one graph.
int capture(skycell_plan *p, const void *points, int32_t *out_idx, int32_t *out_count)
{
    drop_graph(p);
    const size_t esize = p->dtype == SKYCELL_DTYPE_F32 ? 4 : 2;
    const int kBranches = batch_branches();
    std::lock_guard<std::mutex> lk(g_kit_mu);
    CaptureKit *kit = nullptr;
    hipError_t e = capture_kit(p->device, &kit);
    if (e != hipSuccess) return set_error(SKYCELL_E_HIP, "creating capture streams: %s", hipGetErrorString(e));
    hipStream_t origin = kit->origin;
    hipStream_t *branch = kit->branch;
    hipEvent_t fork = kit->fork, *join = kit->join;
    int rc = SKYCELL_OK;
    bool capturing = false;
    if (e == hipSuccess) e = hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        capturing = true;
        e = hipEventRecord(fork, origin);
        for (int i = 0; i < kBranches && e == hipSuccess; ++i) e = hipStreamWaitEvent(branch[i], fork, 0);
    }
    for (int32_t s = 0; s < p->num_inst && e == hipSuccess && rc == SKYCELL_OK; ++s) {
        const uint32_t b = p->order[s];
        hipStream_t st = branch[s % kBranches];
        if (p->n[b] == 0) {
            e = launch_write_zero_count(out_count + b, st);
            continue;
        }
        rc = run_pipeline((const char *)points + (size_t)p->pts_off[b] * esize, p->dtype, p->n[b], p->d[b],
                          p->g[b], p->value_bits, out_idx + p->out_off[b], out_count + b, p->d_ws + p->ws_off[b],
                          nullptr, st);
    }
    // join every branch even after an error, so that the capture ends cleanly
    // and the (reused) branch streams leave capture mode
    for (int i = 0; i < kBranches && capturing; ++i) {
        hipError_t ej = hipEventRecord(join[i], branch[i]);
        if (ej == hipSuccess) ej = hipStreamWaitEvent(origin, join[i], 0);
        if (e == hipSuccess) e = ej;
    }
    if (capturing) {
        const hipError_t ee = hipStreamEndCapture(origin, &p->graph);
        if (e == hipSuccess) e = ee;
    }
    if (e == hipSuccess && rc == SKYCELL_OK) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (rc != SKYCELL_OK || e != hipSuccess) {
        drop_graph(p);
        return rc != SKYCELL_OK ? rc : set_error(SKYCELL_E_HIP, "capturing the batch: %s", hipGetErrorString(e));
    }
    p->bound_points = points;
    p->bound_out_idx = out_idx;
    p->bound_out_count = out_count;
    return SKYCELL_OK;
}

}  // namespace

extern "C" {

int skycell_batched_plan_create(int32_t num_inst, const int64_t *h_n, const int32_t *h_d, int32_t dtype,
                                int32_t value_bits, const int32_t *h_grid, skycell_plan_t *plan)
{
    if (plan == nullptr) return set_error(SKYCELL_E_INVAL, "plan is NULL");
    *plan = nullptr;
    if (num_inst < 1) return set_error(SKYCELL_E_INVAL, "num_inst = %d must be >= 1", num_inst);
    if (h_n == nullptr || h_d == nullptr) return set_error(SKYCELL_E_INVAL, "n or d array is NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return set_error(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    if (value_bits < 1 || value_bits > 16) return set_error(SKYCELL_E_RANGE, "value_bits = %d outside [1, 16]", value_bits);

    skycell_plan *p = new skycell_plan();
    p->dtype = dtype;
    p->value_bits = value_bits;
    p->num_inst = num_inst;
    p->n.assign(h_n, h_n + num_inst);
    p->d.assign(h_d, h_d + num_inst);
    p->g.assign(num_inst, 1);
    p->pts_off.assign(num_inst + 1, 0);
    p->out_off.assign(num_inst + 1, 0);
    p->ws_off.assign(num_inst + 1, 0);
    for (int32_t b = 0; b < num_inst; ++b) {
        if (h_n[b] < 0 || h_n[b] >= ((int64_t)1 << 31)) {
            plan_free(p);
            return set_error(SKYCELL_E_INVAL, "instance %d: n = %lld out of range", b, (long long)h_n[b]);
        }
        if (h_d[b] < 1 || h_d[b] > SKYCELL_MAX_D) {
            plan_free(p);
            return set_error(SKYCELL_E_INVAL, "instance %d: d = %d outside [1, %d]", b, h_d[b], SKYCELL_MAX_D);
        }
        if (h_grid != nullptr && h_grid[b] < 0) {
            plan_free(p);
            return set_error(SKYCELL_E_INVAL, "instance %d: grid_res < 0", b);
        }
        const int g = (h_grid != nullptr && h_grid[b] > 0) ? h_grid[b] : choose_grid_batched(h_n[b], h_d[b], dtype);
        if (grid_cells(g, h_d[b]) > batch_max_cells(h_n[b])) {
            plan_free(p);
            return set_error(SKYCELL_E_RANGE, "instance %d: %d columns in %d dimensions exceed %llu cells", b, g,
                             h_d[b], (unsigned long long)batch_max_cells(h_n[b]));
        }
        p->g[b] = g;
        p->pts_off[b + 1] = p->pts_off[b] + h_n[b] * h_d[b];
        p->out_off[b + 1] = p->out_off[b] + h_n[b];
        const size_t ws = h_n[b] > 0 ? workspace_layout(h_n[b], h_d[b], grid_desc(h_d[b], p->g[b]).cells, nullptr, nullptr) : 0;
        p->ws_off[b + 1] = p->ws_off[b] + ws;
    }
    if (p->out_off[num_inst] >= ((int64_t)1 << 31)) {
        plan_free(p);
        return set_error(SKYCELL_E_RANGE, "batch holds 2^31 points or more");
    }
    // every instance's slices lie inside the batch totals
    for (int32_t b = 0; b < num_inst; ++b) {
        if (p->pts_off[b] + p->n[b] * p->d[b] > p->pts_off[num_inst] || p->out_off[b] + p->n[b] > p->out_off[num_inst] ||
            p->ws_off[b] > p->ws_off[num_inst]) {
            plan_free(p);
            return set_error(SKYCELL_E_INVAL, "instance %d: inconsistent batch layout", b);
        }
    }
    p->order.resize(num_inst);
    std::iota(p->order.begin(), p->order.end(), 0u);
    std::stable_sort(p->order.begin(), p->order.end(), [&](uint32_t a, uint32_t b) {
        return (double)h_n[a] * h_d[a] * h_d[a] > (double)h_n[b] * h_d[b] * h_d[b];
    });

    hipError_t e = hipGetDevice(&p->device);
    if (e == hipSuccess) e = hipMalloc(&p->d_ws, std::max<size_t>(p->ws_off[num_inst], 256));
    if (e != hipSuccess) {
        const size_t bytes = p->ws_off[num_inst];
        plan_free(p);
        return set_error(SKYCELL_E_NOMEM, "plan workspace of %zu bytes: %s", bytes, hipGetErrorString(e));
    }
    // resolve the host-side queries of every launch before any capture
    for (int32_t b = 0; b < num_inst; ++b) {
        if ((e = refine_prepare(pipeline_desc(h_n[b], h_d[b], p->g[b], dtype))) != hipSuccess) {
            plan_free(p);
            return set_error(SKYCELL_E_HIP, "preparing instance %d: %s", b, hipGetErrorString(e));
        }
    }
    (void)device_cus(p->device);
    *plan = p;
    return clear_error();
}

int skycell_batched_offsets(skycell_plan_t plan, int64_t *points_off, int64_t *out_off, int32_t *grid_res)
{
    if (plan == nullptr) return set_error(SKYCELL_E_INVAL, "plan is NULL");
    for (int32_t b = 0; b <= plan->num_inst; ++b) {
        if (points_off) points_off[b] = plan->pts_off[b];
        if (out_off) out_off[b] = plan->out_off[b];
        if (grid_res && b < plan->num_inst) grid_res[b] = plan->g[b];
    }
    return clear_error();
}

int skycell_batched_run(skycell_plan_t plan, const void *points, int32_t *out_idx, int32_t *out_count,
                        void *stream)
{
    if (plan == nullptr) return set_error(SKYCELL_E_INVAL, "plan is NULL");
    if (out_count == nullptr) return set_error(SKYCELL_E_INVAL, "out_count is NULL");
    if (plan->out_off[plan->num_inst] > 0 && (points == nullptr || out_idx == nullptr))
        return set_error(SKYCELL_E_INVAL, "points or out_idx is NULL");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return set_error(SKYCELL_E_HIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev != plan->device) return set_error(SKYCELL_E_INVAL, "plan was created on device %d, current is %d", plan->device, dev);
    if (plan->exec == nullptr || points != plan->bound_points || out_idx != plan->bound_out_idx ||
        out_count != plan->bound_out_count) {
        const int rc = capture(plan, points, out_idx, out_count);
        if (rc != SKYCELL_OK) return rc;
    }
    if ((e = hipGraphLaunch(plan->exec, (hipStream_t)stream)) != hipSuccess)
        return set_error(SKYCELL_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
    if (plan->launched == nullptr &&
        (e = hipEventCreateWithFlags(&plan->launched, hipEventDisableTiming)) != hipSuccess) {
        plan->launched = nullptr;
        return set_error(SKYCELL_E_HIP, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if ((e = hipEventRecord(plan->launched, (hipStream_t)stream)) != hipSuccess)
        return set_error(SKYCELL_E_HIP, "hipEventRecord: %s", hipGetErrorString(e));
    plan->launched_pending = true;
    return clear_error();
}

int skycell_plan_destroy(skycell_plan_t plan)
{
    if (plan == nullptr) return set_error(SKYCELL_E_INVAL, "plan is NULL");
    (void)hipDeviceSynchronize();
    plan_free(plan);
    return clear_error();
}

}  // extern "C"
