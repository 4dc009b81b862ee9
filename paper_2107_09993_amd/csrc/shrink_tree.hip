// The paper's parallel ShrinkKeyCells (Section V-B, Algorithm 3) driven layer by
// layer as in Algorithm 1, as an alternative to the prefix-OR cell prune.
//
// Layer 0 is one cell, a key and candidate cell.  For i = 0 .. rho-1 the leaves
// of a complete binary tree are the 2^d children of every candidate cell of
// layer i (key cells included), empty ones too.  For each rotation m = 0 ..
// d-2 the leaves are put in order of their columns under the rotation
// (rotated dimension k is dimension (k + m) mod d; rotated dimension d-1 most
// significant); a bottom-up sweep sets u of a node to dom_2 of its children's
// u, a top-down sweep sets l from the node's own u and the l of the node left
// of its parent; after the last rotation a leaf is a key cell when l = o, a
// candidate when l partially dominates o, dominated when l dominates o.
// Layer i+1's candidate cells (key cells included) seed the next layer.
//
// dom_2(a, b) returns a when cell a holds points, a <= b in every dimension,
// and a equals b in rotated dimensions 2 .. d-1; else b.  A padding leaf loses
// to any cell.  Pointers are Morton indices of the layer's cells (bit b of
// column k at index bit b*d + k), so a leaf's l follows the cell across the
// reorderings of later rotations through the dense array lptr[cell].
//
// What the tree reports is not always what Definition 3 says: with one pointer
// per node a cell that has two incomparable non-empty cells below it can keep
// the one that only partially dominates it, and rotations compare pointers that
// need not agree with the leaf in the fixed dimensions.  Its "dominated"
// verdicts are always right (the pointer it holds dominates the cell), so the
// cells it keeps are a superset of Definition 3's survivors and the refine
// still gives the exact skyline; it only prunes less.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <new>
#include <vector>

#include "../../include/skycell.h"
#include "cellops.h"
#include "common.h"
#include "host_internal.h"
#include "scan.h"

namespace skycell {

constexpr int kTreeThreads = 256;
constexpr uint32_t kPad = 0xFFFFFFFFu;

static inline dim3 tree_grid(uint64_t count)
{
    uint64_t b = (count + kTreeThreads - 1) / kTreeThreads;
    return dim3((unsigned)(b ? b : 1));
}

__device__ __forceinline__ bool bit_of(const uint64_t *bits, uint32_t x) { return (bits[x >> 6] >> (x & 63)) & 1ull; }

// Column k of a Morton index of a layer with L bits per column.
__device__ __forceinline__ uint32_t col_of(uint32_t x, int k, int d, int L)
{
    uint32_t c = 0u;
    for (int b = 0; b < L; ++b) c |= ((x >> (b * d + k)) & 1u) << b;
    return c;
}

struct TreeLayer {
    int d, L, m;             // dimensions, bits per column, rotation
    const uint64_t *occ;     // occupancy of the layer, one bit per cell
};

__device__ __forceinline__ uint32_t dom2(const TreeLayer &t, uint32_t a, uint32_t b)
{
    if (a == kPad) return b;
    if (b == kPad) return a;
    if (!bit_of(t.occ, a)) return b;
    for (int k = 0; k < t.d; ++k) {
        const uint32_t ca = col_of(a, k, t.d, t.L), cb = col_of(b, k, t.d, t.L);
        if (ca > cb) return b;
        const int rk = (k - t.m + t.d) % t.d;  // dimension k's place under the rotation
        if (rk >= 2 && ca != cb) return b;
    }
    return a;
}

// Occupancy of layer rho from the histogram, then of each coarser layer: bit x
// of layer j is the OR of bits x * 2^d .. x * 2^d + 2^d - 1 of layer j + 1.
__global__ __launch_bounds__(kTreeThreads) void k_tree_occ_leaf(const uint32_t *__restrict__ cnt, uint32_t cells,
                                                                uint64_t *__restrict__ occ)
{
    const uint32_t x = blockIdx.x * kTreeThreads + threadIdx.x;
    const bool on = x < cells && cnt[x] != 0u;
    const uint64_t b = __ballot(on);
    if (__lane_id() == 0 && x < cells) occ[x >> 6] = b;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_occ_up(const uint64_t *__restrict__ fine, uint32_t coarse_cells,
                                                              int d, uint64_t *__restrict__ coarse)
{
    const uint32_t x = blockIdx.x * kTreeThreads + threadIdx.x;
    bool on = false;
    if (x < coarse_cells) {
        const uint32_t kids = 1u << d;
        const uint64_t first = (uint64_t)x << d;
        if (kids >= 64) {
            for (uint32_t w = 0; w < kids / 64 && !on; ++w) on = fine[(first >> 6) + w] != 0ull;
        } else {
            const uint64_t word = fine[first >> 6];
            const uint64_t mask = ((1ull << kids) - 1ull) << (first & 63);
            on = (word & mask) != 0ull;
        }
    }
    const uint64_t b = __ballot(on);
    if (__lane_id() == 0 && x < coarse_cells) coarse[x >> 6] = b;
}

// Leaves of layer L in the order of rotation m: index t of the rotated
// row-major enumeration -> Morton index of the cell; a leaf when its parent
// (the index without its lowest d bits) is a candidate cell of layer L - 1.
struct LeafLoader {
    int d, L, m;
    const uint64_t *parent_cand;
    __device__ uint32_t cell(uint64_t t) const
    {
        uint32_t x = 0u;
        for (int r = 0; r < d; ++r) {
            const uint32_t c = (uint32_t)(t >> (r * L)) & ((1u << L) - 1u);
            const int k = (r + m) % d;  // rotated dimension r is dimension (r + m) mod d
            for (int b = 0; b < L; ++b) x |= ((c >> b) & 1u) << (b * d + k);
        }
        return x;
    }
    __device__ uint32_t operator()(uint64_t t) const { return bit_of(parent_cand, cell(t) >> d) ? 1u : 0u; }
};

struct LeafEmitter {
    LeafLoader ld;
    uint32_t *leaf;
    __device__ void operator()(uint64_t t, uint32_t prefix, uint32_t v) const
    {
        if (v) leaf[prefix] = ld.cell(t);
    }
};

__global__ void k_tree_count(const uint64_t *block_sums, uint32_t nb, uint32_t *count)
{
    *count = (uint32_t)block_sums[nb];
}

// Level 0 of the tree: u of leaf j (o itself at rotation 0, else the l the
// cell carried out of the previous rotation); padding beyond the leaves.
__global__ __launch_bounds__(kTreeThreads) void k_tree_leaves(const uint32_t *__restrict__ leaf,
                                                              const uint32_t *__restrict__ count, uint32_t size,
                                                              const uint32_t *__restrict__ lptr, int m,
                                                              uint32_t *__restrict__ U)
{
    const uint32_t j = blockIdx.x * kTreeThreads + threadIdx.x;
    if (j >= size) return;
    const uint32_t n = *count;
    U[j] = j < n ? (m == 0 ? leaf[j] : lptr[leaf[j]]) : kPad;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_up(TreeLayer t, const uint32_t *__restrict__ child,
                                                          uint32_t *__restrict__ parent, uint32_t count)
{
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    if (k < count) parent[k] = dom2(t, child[2 * k], child[2 * k + 1]);
}

// Level j of the top-down sweep from level j + 1 (above) and u of level j.
__global__ __launch_bounds__(kTreeThreads) void k_tree_down(TreeLayer t, const uint32_t *__restrict__ Uj,
                                                            const uint32_t *__restrict__ Labove,
                                                            uint32_t *__restrict__ Lj, uint32_t count)
{
    const uint32_t k = blockIdx.x * kTreeThreads + threadIdx.x;
    if (k >= count) return;
    uint32_t l;
    if (k == 0) l = Uj[0];
    else if (k & 1u) l = Labove[(k - 1) >> 1];
    else l = dom2(t, Labove[(k >> 1) - 1], Uj[k]);
    Lj[k] = l;
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_store_l(const uint32_t *__restrict__ leaf,
                                                               const uint32_t *__restrict__ count,
                                                               const uint32_t *__restrict__ L0,
                                                               uint32_t *__restrict__ lptr)
{
    const uint32_t j = blockIdx.x * kTreeThreads + threadIdx.x;
    if (j < *count) lptr[leaf[j]] = L0[j];
}

// Theorem 2 on every leaf: key (l = o, non-empty) and candidate (l partially
// dominates o) cells go into `cand` (and key cells also into `key`).
__global__ __launch_bounds__(kTreeThreads) void k_tree_classify(TreeLayer t, const uint32_t *__restrict__ leaf,
                                                                const uint32_t *__restrict__ count,
                                                                const uint32_t *__restrict__ lptr,
                                                                uint64_t *__restrict__ cand, uint64_t *__restrict__ key)
{
    const uint32_t j = blockIdx.x * kTreeThreads + threadIdx.x;
    if (j >= *count) return;
    const uint32_t o = leaf[j], l = lptr[o];
    bool is_key = false, is_cand = false;
    if (l == o) {
        is_key = bit_of(t.occ, o);
    } else if (l != kPad && bit_of(t.occ, l)) {
        bool le = true, eq = false;
        for (int k = 0; k < t.d; ++k) {
            const uint32_t cl = col_of(l, k, t.d, t.L), co = col_of(o, k, t.d, t.L);
            le &= cl <= co;
            eq |= cl == co;
        }
        is_cand = le && eq;
    }
    if (is_key || is_cand) atomicOr((unsigned long long *)&cand[o >> 6], 1ull << (o & 63));
    if (is_key && key != nullptr) atomicOr((unsigned long long *)&key[o >> 6], 1ull << (o & 63));
}

__global__ __launch_bounds__(kTreeThreads) void k_tree_zero(uint64_t *__restrict__ p, uint64_t words)
{
    for (uint64_t i = (uint64_t)blockIdx.x * kTreeThreads + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * kTreeThreads)
        p[i] = 0ull;
}

__global__ void k_tree_root(uint64_t *cand) { cand[0] = 1ull; }

// Survivors of the tree form: non-empty cells the tree keeps; the record's
// survivor bit and the scatter's bitmap follow them.
__global__ __launch_bounds__(kTreeThreads) void k_tree_apply(const uint64_t *__restrict__ cand,
                                                             const uint32_t *__restrict__ cnt, uint32_t cells,
                                                             uint64_t *__restrict__ rec, uint64_t *__restrict__ survbits,
                                                             uint64_t *__restrict__ stats)
{
    const uint32_t x = blockIdx.x * kTreeThreads + threadIdx.x;
    bool was = false, now = false;
    if (x < cells) {
        const uint64_t r = rec[x];
        was = rec_surv(r);
        now = cnt[x] != 0u && bit_of(cand, x);
        // the count field is kept only for surviving cells (see cell_record)
        const uint32_t c = cnt[x];
        const uint64_t cs = now ? (c < kRecCountSat ? c : kRecCountSat) : 0u;
        rec[x] = (r & ~((1ull << 63) | ((uint64_t)kRecCountSat << 32))) | ((uint64_t)(now ? 1u : 0u) << 63) |
                 (cs << 32);
    }
    const uint64_t bn = __ballot(now), bw = __ballot(was);
    if (__lane_id() == 0 && x < cells) {
        survbits[x >> 6] = bn;
        if (stats != nullptr && bn != bw)
            atomicAdd((unsigned long long *)&stats[SKYCELL_STAT_SURVIVING_CELLS],
                      (unsigned long long)((int64_t)__popcll(bn) - (int64_t)__popcll(bw)));
    }
}

static inline uint64_t words_of(uint64_t cells) { return (cells + 63) / 64; }

size_t tree_scratch_layout(uint32_t cells, int d, int rho, TreeScratch *ts, char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return base ? base + o : nullptr;
    };
    uint64_t occ_words = 0;
    for (int j = 0; j <= rho; ++j) occ_words += words_of((uint64_t)1 << (j * d));
    char *occ = take(occ_words * 8);
    char *c0 = take(words_of(cells) * 8);
    char *c1 = take(words_of(cells) * 8);
    char *leaf = take((size_t)cells * 4);
    char *lptr = take((size_t)cells * 4);
    uint64_t size = 1;
    while (size < cells) size <<= 1;
    char *U = take((size_t)size * 2 * 4);
    char *Lv = take((size_t)size * 2 * 4);
    char *sums = take(((size_t)scan_tiles(cells) + 1) * 8);
    char *count = take(8);
    if (ts) {
        ts->occ = (uint64_t *)occ;
        ts->cand[0] = (uint64_t *)c0;
        ts->cand[1] = (uint64_t *)c1;
        ts->leaf = (uint32_t *)leaf;
        ts->lptr = (uint32_t *)lptr;
        ts->U = (uint32_t *)U;
        ts->Lv = (uint32_t *)Lv;
        ts->sums = (uint64_t *)sums;
        ts->count = (uint32_t *)count;
    }
    return off;
}

// Runs the layers 1..rho; afterwards ts.cand[rho & 1] holds layer rho's
// candidate cells.  With key_out / cand_out (device bitmaps, layer j at word
// offset sum_{i<j} words(2^(i d)) for j >= 1) every layer's key and candidate
// cells are copied out as well.
hipError_t run_shrink_tree(const uint32_t *cnt, int d, int rho, const TreeScratch &ts, uint64_t *key_out,
                           uint64_t *cand_out, hipStream_t st)
{
    const uint32_t cells = 1u << (rho * d);
    std::vector<uint64_t> occ_off((size_t)rho + 2, 0);
    for (int j = 0; j <= rho; ++j) occ_off[j + 1] = occ_off[j] + words_of((uint64_t)1 << (j * d));
    hipLaunchKernelGGL(k_tree_occ_leaf, tree_grid(cells), dim3(kTreeThreads), 0, st, cnt, cells, ts.occ + occ_off[rho]);
    for (int j = rho - 1; j >= 0; --j) {
        const uint32_t cc = 1u << (j * d);
        hipLaunchKernelGGL(k_tree_occ_up, tree_grid(cc), dim3(kTreeThreads), 0, st,
                           (const uint64_t *)(ts.occ + occ_off[j + 1]), cc, d, ts.occ + occ_off[j]);
    }
    hipLaunchKernelGGL(k_tree_zero, dim3(1), dim3(kTreeThreads), 0, st, ts.cand[0], (uint64_t)1);
    hipLaunchKernelGGL(k_tree_root, dim3(1), dim3(1), 0, st, ts.cand[0]);
    uint64_t out_off = 0;
    const int rotations = d > 1 ? d - 1 : 1;
    for (int L = 1; L <= rho; ++L) {
        const uint32_t lcells = 1u << (L * d);
        const uint64_t *parent = ts.cand[(L - 1) & 1];
        uint64_t *cur = ts.cand[L & 1];
        hipLaunchKernelGGL(k_tree_zero, dim3(std::min<unsigned>(1024u, tree_grid(words_of(lcells)).x)),
                           dim3(kTreeThreads), 0, st, cur, words_of(lcells));
        // every leaf count fits: leaves = 2^d * candidates <= the layer's cells
        uint32_t size = 1;
        while (size < lcells) size <<= 1;
        int h = 0;
        while ((1u << h) < size) ++h;
        for (int m = 0; m < rotations; ++m) {
            const TreeLayer t{d, L, m, ts.occ + occ_off[L]};
            LeafLoader ld{d, L, m, parent};
            LeafEmitter em{ld, ts.leaf};
            hipError_t e = enqueue_scan<uint32_t>(ld, em, lcells, ts.sums, st);
            if (e != hipSuccess) return e;
            hipLaunchKernelGGL(k_tree_count, dim3(1), dim3(1), 0, st, (const uint64_t *)ts.sums, scan_tiles(lcells),
                               ts.count);
            // level j of U and Lv occupies [lvl[j], lvl[j] + (size >> j)), lvl[0] = 0
            hipLaunchKernelGGL(k_tree_leaves, tree_grid(size), dim3(kTreeThreads), 0, st, (const uint32_t *)ts.leaf,
                               (const uint32_t *)ts.count, size, (const uint32_t *)ts.lptr, m, ts.U);
            uint64_t base = 0;
            std::vector<uint64_t> lvl((size_t)h + 1);
            for (int j = 0; j <= h; ++j) {
                lvl[j] = base;
                base += size >> j;
            }
            for (int j = 1; j <= h; ++j) {
                const uint32_t c = size >> j;
                hipLaunchKernelGGL(k_tree_up, tree_grid(c), dim3(kTreeThreads), 0, st, t,
                                   (const uint32_t *)(ts.U + lvl[j - 1]), ts.U + lvl[j], c);
            }
            // top level: l = u
            hipLaunchKernelGGL(k_tree_down, dim3(1), dim3(kTreeThreads), 0, st, t, (const uint32_t *)(ts.U + lvl[h]),
                               (const uint32_t *)(ts.Lv + lvl[h]), ts.Lv + lvl[h], 1u);
            for (int j = h - 1; j >= 0; --j) {
                const uint32_t c = size >> j;
                hipLaunchKernelGGL(k_tree_down, tree_grid(c), dim3(kTreeThreads), 0, st, t,
                                   (const uint32_t *)(ts.U + lvl[j]), (const uint32_t *)(ts.Lv + lvl[j + 1]),
                                   ts.Lv + lvl[j], c);
            }
            hipLaunchKernelGGL(k_tree_store_l, tree_grid(size), dim3(kTreeThreads), 0, st, (const uint32_t *)ts.leaf,
                               (const uint32_t *)ts.count, (const uint32_t *)ts.Lv, ts.lptr);
        }
        const TreeLayer t{d, L, rotations - 1, ts.occ + occ_off[L]};
        uint64_t *key = key_out ? key_out + out_off : nullptr;
        if (key_out) {
            hipLaunchKernelGGL(k_tree_zero, dim3(std::min<unsigned>(1024u, tree_grid(words_of(lcells)).x)),
                               dim3(kTreeThreads), 0, st, key, words_of(lcells));
        }
        hipLaunchKernelGGL(k_tree_classify, tree_grid(size), dim3(kTreeThreads), 0, st, t, (const uint32_t *)ts.leaf,
                           (const uint32_t *)ts.count, (const uint32_t *)ts.lptr, cur, key);
        if (cand_out) {
            hipError_t e = hipMemcpyAsync(cand_out + out_off, cur, words_of(lcells) * 8, hipMemcpyDeviceToDevice, st);
            if (e != hipSuccess) return e;
        }
        out_off += words_of(lcells);
    }
    return hipGetLastError();
}

hipError_t apply_shrink_tree(const TreeScratch &ts, int rho, const Workspace &ws, uint32_t cells, uint64_t *stats,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_tree_apply, tree_grid(cells), dim3(kTreeThreads), 0, st, (const uint64_t *)ts.cand[rho & 1],
                       (const uint32_t *)ws.cnt, cells, ws.rec, ws.survbits, stats);
    return hipGetLastError();
}

}  // namespace skycell

using namespace skycell;

int skycell_shrink_tree(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t rho, int32_t value_bits,
                        uint64_t *key_out, uint64_t *cand_out, void *stream)
{
    if (points == nullptr && n > 0) return set_error(SKYCELL_E_INVAL, "points is NULL");
    if (key_out == nullptr || cand_out == nullptr) return set_error(SKYCELL_E_INVAL, "an output is NULL");
    if (dtype != SKYCELL_DTYPE_F32 && dtype != SKYCELL_DTYPE_U16)
        return set_error(SKYCELL_E_INVAL, "dtype %d is not SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16", dtype);
    if (n < 1 || n >= (int64_t)1 << 31) return set_error(SKYCELL_E_INVAL, "n = %lld is outside [1, 2^31)", (long long)n);
    if (d < 1 || d > SKYCELL_MAX_D) return set_error(SKYCELL_E_INVAL, "d = %d is outside [1, %d]", d, SKYCELL_MAX_D);
    if (rho < 1 || rho * d > 26) return set_error(SKYCELL_E_RANGE, "rho = %d: need 1 <= rho and rho * d <= 26", rho);
    if (dtype == SKYCELL_DTYPE_F32) value_bits = 16;
    if (value_bits < 1 || value_bits > 16) return set_error(SKYCELL_E_RANGE, "value_bits = %d outside [1, 16]", value_bits);
    hipStream_t st = (hipStream_t)stream;
    const int g = 1 << rho;
    const GridDesc gd = grid_desc(d, g);
    int dev = 0;
    SKYCELL_HIP_CHECK(hipGetDevice(&dev));
    const size_t wneed = workspace_layout(n, d, gd.cells, nullptr, nullptr);
    const size_t tneed = tree_scratch_layout(gd.cells, d, rho, nullptr, nullptr);
    void *wptr = nullptr, *tptr = nullptr;
    int rc = cached_buffer(kCacheWorkspace, dev, st, wneed, &wptr);
    if (rc != SKYCELL_OK) return rc;
    if ((rc = cached_buffer(kCacheTree, dev, st, tneed, &tptr)) != SKYCELL_OK) return rc;
    Workspace ws;
    workspace_layout(n, d, gd.cells, &ws, (char *)wptr);
    TreeScratch ts;
    tree_scratch_layout(gd.cells, d, rho, &ts, (char *)tptr);
    SKYCELL_HIP_CHECK(launch_init(ws, gd, nullptr, st));
    SKYCELL_HIP_CHECK(launch_quantize_hist(points, dtype, n, gd, value_bits, ws, st));
    SKYCELL_HIP_CHECK(run_shrink_tree(ws.cnt, d, rho, ts, key_out, cand_out, st));
    return clear_error();
}
