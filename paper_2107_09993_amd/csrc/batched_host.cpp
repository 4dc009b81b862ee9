// C ABI of the batched path: plan creation (instance layout, grid choice,
// workspace, one captured hipGraph holding the persistent launch), runs and
// destruction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <numeric>
#include <vector>

#include "../../include/skycell.h"
#include "batched.h"
#include "common.h"
#include "host_internal.h"

using namespace skycell;

struct skycell_plan {
    int device = 0;
    int dtype = SKYCELL_DTYPE_F32;
    int value_bits = 16;
    uint32_t num_inst = 0;
    uint32_t num_chunks = 0;
    uint32_t chunk_items = 0;
    unsigned blocks = 0;
    std::vector<BatchInst> inst;
    std::vector<int64_t> pts_off;  // [num_inst + 1] element offsets
    std::vector<int64_t> out_off;  // [num_inst + 1]
    BatchInst *d_inst = nullptr;
    uint32_t *d_prep_order = nullptr;
    uint32_t *d_chunk_inst = nullptr;
    uint32_t *d_ctl = nullptr;
    uint32_t *d_ictl = nullptr;
    char *d_ws = nullptr;
    size_t ws_bytes = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    const void *bound_points = nullptr;
    int32_t *bound_out_idx = nullptr;
    int32_t *bound_out_count = nullptr;
};

namespace {

constexpr uint32_t kChunkItems = 256;
constexpr uint32_t kBatchMaxCells = 1u << 20;

void plan_free(skycell_plan *p)
{
    if (p == nullptr) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    for (void *q : {(void *)p->d_inst, (void *)p->d_prep_order, (void *)p->d_chunk_inst, (void *)p->d_ctl,
                    (void *)p->d_ictl, (void *)p->d_ws})
        if (q) (void)hipFree(q);
    delete p;
}

void drop_graph(skycell_plan *p)
{
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
    p->bound_points = nullptr;
    p->bound_out_idx = nullptr;
    p->bound_out_count = nullptr;
}

// Capture the persistent launch with this run's buffers as its arguments into
// a one-node graph and instantiate it.  The graph is kept and replayed while
// later runs pass the same buffers.
hipError_t capture(skycell_plan *p, const void *points, int32_t *out_idx, int32_t *out_count)
{
    drop_graph(p);
    BatchLaunch L;
    memset(&L, 0, sizeof(L));
    L.dtype = p->dtype;
    L.points = points;
    L.inst = p->d_inst;
    L.prep_order = p->d_prep_order;
    L.num_inst = p->num_inst;
    L.chunk_inst = p->d_chunk_inst;
    L.num_chunks = p->num_chunks;
    L.chunk_items = p->chunk_items;
    L.ctl = p->d_ctl;
    L.ictl = p->d_ictl;
    L.out_idx = out_idx;
    L.out_count = out_count;
    L.value_bits = p->value_bits;
    L.blocks = p->blocks;
    hipStream_t cs = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        const hipError_t le = launch_batched(L, cs);
        e = hipStreamEndCapture(cs, &p->graph);
        if (e == hipSuccess) e = le;
    }
    (void)hipStreamDestroy(cs);
    if (e == hipSuccess) e = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        drop_graph(p);
        return e;
    }
    p->bound_points = points;
    p->bound_out_idx = out_idx;
    p->bound_out_count = out_count;
    return hipSuccess;
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

    std::vector<int> g(num_inst);
    int64_t total_out = 0;
    for (int32_t b = 0; b < num_inst; ++b) {
        if (h_n[b] < 0 || h_n[b] >= ((int64_t)1 << 31))
            return set_error(SKYCELL_E_INVAL, "instance %d: n = %lld out of range", b, (long long)h_n[b]);
        if (h_d[b] < 1 || h_d[b] > SKYCELL_MAX_D)
            return set_error(SKYCELL_E_INVAL, "instance %d: d = %d outside [1, %d]", b, h_d[b], SKYCELL_MAX_D);
        g[b] = (h_grid != nullptr && h_grid[b] > 0) ? h_grid[b] : choose_grid_batched(h_n[b], h_d[b], dtype);
        if (h_grid != nullptr && h_grid[b] < 0) return set_error(SKYCELL_E_INVAL, "instance %d: grid_res < 0", b);
        if (grid_cells(g[b], h_d[b]) > kBatchMaxCells)
            return set_error(SKYCELL_E_RANGE, "instance %d: %d columns in %d dimensions exceed %u cells", b, g[b],
                             h_d[b], kBatchMaxCells);
        total_out += h_n[b];
    }
    if (total_out >= ((int64_t)1 << 31)) return set_error(SKYCELL_E_RANGE, "batch holds 2^31 points or more");

    skycell_plan *p = new skycell_plan();
    p->dtype = dtype;
    p->value_bits = value_bits;
    p->num_inst = (uint32_t)num_inst;
    p->chunk_items = kChunkItems;
    p->inst.resize(num_inst);
    p->pts_off.assign(num_inst + 1, 0);
    p->out_off.assign(num_inst + 1, 0);
    std::vector<size_t> ws_off(num_inst + 1, 0);
    for (int32_t b = 0; b < num_inst; ++b) {
        const GridDesc gd = grid_desc(h_d[b], g[b]);
        p->pts_off[b + 1] = p->pts_off[b] + h_n[b] * h_d[b];
        p->out_off[b + 1] = p->out_off[b] + h_n[b];
        ws_off[b + 1] = ws_off[b] + workspace_layout(h_n[b], h_d[b], gd.cells, nullptr, nullptr);
    }
    p->ws_bytes = ws_off[num_inst];

    // largest estimated work first: stage A order and chunk order
    std::vector<uint32_t> order(num_inst);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return (double)h_n[a] * h_d[a] * h_d[a] > (double)h_n[b] * h_d[b] * h_d[b];
    });
    std::vector<uint32_t> chunk_inst;
    std::vector<uint32_t> chunk0(num_inst), nch(num_inst);
    for (uint32_t b : order) {
        const uint32_t c = std::max<uint32_t>(1u, (uint32_t)((h_n[b] + kChunkItems - 1) / kChunkItems));
        chunk0[b] = (uint32_t)chunk_inst.size();
        nch[b] = c;
        chunk_inst.insert(chunk_inst.end(), c, b);
    }
    p->num_chunks = (uint32_t)chunk_inst.size();

    auto fail_free = [&](int code, const char *what, hipError_t e) {
        plan_free(p);
        return set_error(code, "%s: %s", what, hipGetErrorString(e));
    };
    hipError_t e;
    if ((e = hipGetDevice(&p->device)) != hipSuccess) return fail_free(SKYCELL_E_HIP, "hipGetDevice", e);
    if ((e = hipMalloc(&p->d_ws, std::max<size_t>(p->ws_bytes, 256))) != hipSuccess)
        return fail_free(SKYCELL_E_NOMEM, "workspace allocation", e);
    for (int32_t b = 0; b < num_inst; ++b) {
        BatchInst &I = p->inst[b];
        memset(&I, 0, sizeof(I));
        I.pts_off = (uint64_t)p->pts_off[b];
        I.n = (uint32_t)h_n[b];
        I.out_off = (uint32_t)p->out_off[b];
        I.chunk0 = chunk0[b];
        I.nchunks = nch[b];
        I.gd = grid_desc(h_d[b], g[b]);
        Workspace w;
        workspace_layout(h_n[b], h_d[b], I.gd.cells, &w, p->d_ws + ws_off[b]);
        I.cell_of = w.cell_of;
        I.rank = w.rank;
        I.cnt = w.cnt;
        I.lc = w.lc;
        I.rec = w.rec;
        I.keys = w.keys;
        I.fkeys = w.fkeys;
        I.sidx = w.sidx;
        I.items = w.items;
        I.flag = w.flag;
    }
    if ((e = hipMalloc(&p->d_inst, sizeof(BatchInst) * num_inst)) != hipSuccess ||
        (e = hipMalloc(&p->d_prep_order, 4 * (size_t)num_inst)) != hipSuccess ||
        (e = hipMalloc(&p->d_chunk_inst, 4 * (size_t)p->num_chunks)) != hipSuccess ||
        (e = hipMalloc(&p->d_ctl, 4 * (size_t)kBatchCtlWords)) != hipSuccess ||
        (e = hipMalloc(&p->d_ictl, 4 * (size_t)kInstWords * num_inst)) != hipSuccess)
        return fail_free(SKYCELL_E_NOMEM, "plan allocation", e);
    if ((e = hipMemcpy(p->d_inst, p->inst.data(), sizeof(BatchInst) * num_inst, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_prep_order, order.data(), 4 * (size_t)num_inst, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemcpy(p->d_chunk_inst, chunk_inst.data(), 4 * (size_t)p->num_chunks, hipMemcpyHostToDevice)) != hipSuccess ||
        (e = hipMemset(p->d_ctl, 0, 4 * (size_t)kBatchCtlWords)) != hipSuccess ||
        (e = hipMemset(p->d_ictl, 0, 4 * (size_t)kInstWords * num_inst)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
        return fail_free(SKYCELL_E_HIP, "plan upload", e);

    p->blocks = (unsigned)(device_cus(p->device) * batched_blocks_per_cu(dtype));

    *plan = p;
    return clear_error();
}

int skycell_batched_offsets(skycell_plan_t plan, int64_t *points_off, int64_t *out_off, int32_t *grid_res)
{
    if (plan == nullptr) return set_error(SKYCELL_E_INVAL, "plan is NULL");
    for (uint32_t b = 0; b <= plan->num_inst; ++b) {
        if (points_off) points_off[b] = plan->pts_off[b];
        if (out_off) out_off[b] = plan->out_off[b];
        if (grid_res && b < plan->num_inst) grid_res[b] = plan->inst[b].gd.g;
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
        if ((e = capture(plan, points, out_idx, out_count)) != hipSuccess)
            return set_error(SKYCELL_E_HIP, "capturing the batched launch: %s", hipGetErrorString(e));
    }
    if ((e = hipGraphLaunch(plan->exec, (hipStream_t)stream)) != hipSuccess)
        return set_error(SKYCELL_E_HIP, "hipGraphLaunch: %s", hipGetErrorString(e));
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
