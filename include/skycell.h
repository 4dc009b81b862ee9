/*
 * skycell.h -- C ABI of the MI355X (gfx950) exact-skyline library.
 *
 * The library computes the skyline of n points in d attributes (SkyCell paper,
 * Section III, Definitions 1-2): point p dominates q iff p[k] <= q[k] in every
 * dimension and p[l] < q[l] in at least one; the skyline is the set of points no
 * other point dominates.  Smaller is better.  The result is exact and unique; it
 * is returned as ascending int32 indices, every exact copy of a skyline point
 * included (copies never dominate each other).
 *
 * Method (Section V, Algorithm 1, single grid layer): points are mapped to a
 * regular grid of g cells per dimension (Equation 1); cells dominated by a
 * non-empty cell (Definition 3: smaller column in every dimension) are pruned,
 * since they cannot hold skyline points; each remaining point is then checked
 * for point domination against the points of the non-empty cells in its lower
 * cone (cells whose columns are <= its own in every dimension), which is the
 * only place a dominator can sit.
 *
 * Conventions shared by every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller.  Work is enqueued
 *     on `stream` (a hipStream_t passed as void*, NULL = default stream) and runs
 *     asynchronously: the caller keeps inputs alive and reads outputs only after
 *     the stream has passed this call.
 *   - `points` is structure-of-arrays: attribute k of point i is points[k*n + i].
 *   - `out_idx` needs capacity n; `out_idx[0 .. *out_count)` receives the skyline
 *     indices in ascending order.  `*out_count` is written on the device; a
 *     negative value there is a device-detected error (SKYCELL_E_NAN).
 *   - The return value is SKYCELL_OK or a negative code, decided on the host.
 *     All argument checks happen before any HIP call, so they also work on a
 *     machine without a GPU.  skycell_last_error() describes the last failure
 *     of the calling thread.  No C++ exception crosses this interface.
 *   - The result never depends on grid_res, on the autotuner or on tuning.
 */
#ifndef SKYCELL_H
#define SKYCELL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    SKYCELL_OK = 0,
    SKYCELL_E_INVAL = -1, /* null pointer, n < 0, n >= 2^31, d outside [1, 16], bad enum  */
    SKYCELL_E_RANGE = -2, /* cell index space exceeds SKYCELL_MAX_CELLS, bad value_bits    */
    SKYCELL_E_NOMEM = -3, /* device allocation failed, or workspace smaller than required  */
    SKYCELL_E_HIP = -4,   /* a HIP runtime call or kernel launch failed                    */
    SKYCELL_E_NODEV = -5, /* no usable GPU                                                 */
    SKYCELL_E_NAN = -6    /* written to *out_count when the input holds a NaN              */
    /* SKYCELL_E_RANGE is also written to *out_count when a pivot index is outside [0, n)   */
};

#define SKYCELL_MAX_D 16
#define SKYCELL_MAX_CELLS (1u << 26)

#define SKYCELL_DTYPE_F32 0
#define SKYCELL_DTYPE_U16 1

/* Number of uint64 counters written by the *_stats variants (device memory). */
#define SKYCELL_NUM_STATS 9
/* Indices into the stats array.                                               */
#define SKYCELL_STAT_NONEMPTY_CELLS 0  /* cells holding at least one point           */
#define SKYCELL_STAT_SURVIVING_CELLS 1 /* non-empty cells not dominated (Def. 3)     */
#define SKYCELL_STAT_SURVIVOR_POINTS 2 /* points in surviving cells                  */
#define SKYCELL_STAT_ITEMS 3           /* refine work items (groups of query points) */
#define SKYCELL_STAT_CELL_VISITS 4     /* lower-cone cells visited by the refine     */
#define SKYCELL_STAT_PAIR_TESTS 5      /* candidate x query point domination tests   */
#define SKYCELL_STAT_SKYLINE 6         /* number of skyline points                   */
#define SKYCELL_STAT_GRID_RES 7        /* cells per dimension used                   */
#define SKYCELL_STAT_PIVOT_REMOVED 8   /* points of surviving cells a pivot dominates
                                          (pivoted calls; 0 otherwise)               */

/*
 * Exact skyline of binary32 points (Definitions 1-2).
 *   points    device, SoA [d][n] binary32.  Any finite value or +-inf is accepted
 *             (values outside [0, 1) land in the border cells, Equation 1 with a
 *             clamp); -0.0 equals +0.0; a NaN makes *out_count = SKYCELL_E_NAN.
 *   n         number of points, 0 <= n < 2^31.  n = 0 writes *out_count = 0.
 *   d         number of attributes, 1 <= d <= SKYCELL_MAX_D.
 *   grid_res  cells per dimension g >= 1 (the paper uses g = 2^rho, Section III);
 *             0 lets the library choose (skycell_choose_grid).  Cells are
 *             numbered in Morton order over r = ceil(log2 g) bits per dimension,
 *             so 2^(r*d) must not exceed SKYCELL_MAX_CELLS.
 *   out_idx   device int32 [n], written.      out_count  device int32 [1], written.
 *   stream    hipStream_t or NULL.
 * The library keeps a workspace per (device, stream), grown on demand with
 * hipMalloc; use skycell_compute_ws to supply it instead.
 */
int skycell_compute(const float *points, int64_t n, int32_t d, int32_t grid_res,
                    int32_t *out_idx, int32_t *out_count, void *stream);

/*
 * Same for unsigned 16-bit attributes (integer-valued data with many ties).
 *   value_bits  values are expected below 2^value_bits (1..16); the column of v
 *               is floor(v * g / 2^value_bits), clamped to g-1.  Larger values
 *               stay exact but land in the top cell.
 */
int skycell_compute_u16(const uint16_t *points, int64_t n, int32_t d, int32_t grid_res,
                        int32_t value_bits, int32_t *out_idx, int32_t *out_count, void *stream);

/*
 * Workspace size in bytes for skycell_compute_ws with these arguments.
 *   dtype  SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16.  grid_res 0 = autotuned.
 */
int skycell_workspace_bytes(int64_t n, int32_t d, int32_t grid_res, int32_t dtype,
                            size_t *bytes);

/*
 * Exact skyline with a caller-supplied workspace: no allocation happens inside.
 *   points      device SoA [d][n], binary32 (dtype F32) or uint16 (dtype U16).
 *   value_bits  used for U16 only (see skycell_compute_u16).
 *   workspace   device memory of at least skycell_workspace_bytes(...) bytes,
 *               256-byte aligned; its contents are scratch for this call only.
 *               Two calls that overlap in time must not share a workspace.
 *   stats       NULL, or device uint64 [SKYCELL_NUM_STATS] receiving the
 *               counters listed above (this adds a few atomics per wave).
 */
int skycell_compute_ws(const void *points, int32_t dtype, int64_t n, int32_t d,
                       int32_t grid_res, int32_t value_bits, int32_t *out_idx,
                       int32_t *out_count, void *workspace, size_t ws_bytes,
                       uint64_t *stats, void *stream);

/*
 * Exact skyline with a two-layer grid for grids finer than a dense cell table
 * allows (Section III: layer rho has 2^rho columns; a non-empty cell can
 * survive only inside a surviving cell of the layer above).  The base layer,
 * 2^(rho-1) columns, is the dense grid of skycell_compute (histogram, lower
 * closure, records, scatter, refine); the fine layer, 2^rho columns (Equation
 * 1), is kept as one occupancy bit per cell, and its Definition 3 prune is
 * exact: for every surviving base cell, a walk of its lower cone finds which
 * of its fine cells a non-empty fine cell dominates.  Points of dominated fine
 * cells are dropped before the refine.  Same arguments and results as
 * skycell_compute_ws with grid_res replaced by rho; 2 <= d <= 8, rho >= 2,
 * (rho-1)*d <= 26 and rho*d <= 32 (d = 8: g = 16 is 2^32 fine cells).  The
 * library owns the workspace and the two fine bitmaps (2^(rho d) bits each).
 * stats (NULL or device uint64 [SKYCELL_NUM_STATS]): the cell counters count
 * fine cells (non-empty; not dominated inside surviving base cells), the
 * point and refine counters the base path; SKYCELL_STAT_GRID_RES is the base
 * grid.
 */
int skycell_compute_layered(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t rho,
                            int32_t value_bits, int32_t *out_idx, int32_t *out_count, uint64_t *stats,
                            void *stream);

/*
 * For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): skycell_compute_ws
 * without a workspace argument.  Its scratch is a fixed array of
 * SKYCELL_STATIC_SCRATCH_BYTES inside the library, one per GPU, which that GPU
 * holds from the library's first use on it until the process ends; nothing is
 * allocated by this call.  Arguments and results are those of
 * skycell_compute_ws (stats may be NULL).
 *   Size limit: a call whose workspace (skycell_workspace_bytes for the same
 *   n, d, grid_res and dtype) exceeds SKYCELL_STATIC_SCRATCH_BYTES returns
 *   SKYCELL_E_NOMEM before touching the device.
 *   Concurrency: every call on one GPU shares that GPU's array (each call
 *   clears what it needs before use); calls that overlap in time on one GPU,
 *   from any stream or thread, race on it and give undefined results.
 */
#define SKYCELL_STATIC_SCRATCH_BYTES (64u << 20)
int skycell_compute_static(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t grid_res,
                           int32_t value_bits, int32_t *out_idx, int32_t *out_count, uint64_t *stats,
                           void *stream);

/*
 * Grid resolution the library uses when grid_res = 0: the autotuner's entry for
 * d and dtype whose log2 n is nearest to that of n (and at most 1 away) if a
 * tuning table is loaded, else a rule that keeps about one to two cells per
 * point under the cell budget (Section VI: rho <= log(n)/d).
 */
int skycell_choose_grid(int64_t n, int32_t d, int32_t dtype, int32_t *grid_res);

/*
 * Input classes of the tuning table: whether the attributes of the input rise
 * together, trade off against each other, or neither.  The skyline's size and
 * the cost of each grid and refine form depend mostly on this.
 */
#define SKYCELL_CLASS_INDEPENDENT 0
#define SKYCELL_CLASS_CORRELATED 1
#define SKYCELL_CLASS_ANTICORRELATED 2

/*
 * Input class of n points in d attributes (device, SoA [d][n], as for
 * skycell_compute; dtype SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16), from the
 * mean correlation of two attributes over a strided sample of at most 65,536
 * points: > 0.3 correlated, < -0.3/(d-1) anti-correlated, else independent
 * (d = 1: independent).  Enqueued on `stream`, then waits for `stream`: the
 * call returns with *cls set.  Returns SKYCELL_E_INVAL for bad arguments or a
 * stream under graph capture.
 */
int skycell_input_class(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t *cls, void *stream);

/*
 * The configuration a call with grid_res = 0 uses for an input of class cls
 * (-1: not known): grid resolution, refine form (0 lane, 1 wave, as in
 * skycell_set_refine_form) and, for the wave form, waves per item (else 0).
 * Table rows tuned on class cls are preferred, then rows for any class (the
 * lowest mean time over the three classes), then the rules of
 * skycell_choose_grid and skycell_set_refine_form.  skycell_compute and
 * skycell_compute_u16 with grid_res = 0 compute the input's class themselves
 * (skycell_input_class, one synchronisation of the stream) when the table
 * holds class rows for d, dtype and about n, and n >= 65,536.
 */
int skycell_choose_config(int64_t n, int32_t d, int32_t dtype, int32_t cls, int32_t *grid_res, int32_t *form,
                          int32_t *parts);

/*
 * Load an autotuner table (text, one "d log2n dtype g [form [parts [class]]]"
 * line per entry, form 0 = lane, 1 = wave refine, see skycell_set_refine_form;
 * parts the wave form's waves per item, see skycell_set_wave_parts; class the
 * SKYCELL_CLASS_* input class the row was tuned on, absent or -1 for rows
 * chosen over all classes; '#' starts a comment line).  dtype is SKYCELL_DTYPE_* for single calls and
 * SKYCELL_DTYPE_* + 2 for the instances of a batched plan.  NULL clears the
 * table.  Applies to all later calls in the process.  The Python binding loads
 * the table shipped with the package unless SKYCELL_NO_TUNING is set.
 */
int skycell_load_tuning(const char *path);

/*
 * Refine form for all later calls in the process: -1 = chosen per call (the
 * tuning table's form for the call's d, n and grid, else the wave form when
 * the grid has at most n/32 cells), 0 = lane form (one lane walks the lower
 * cone of a few points of one cell; for d <= 8 it passes over every cell whose
 * per-dimension minimum corner rules out its points as dominators), 1 = wave
 * form (one wave walks the cone of up to 63 points of one cell and tests every
 * candidate against all of them), 2 = tile form (grids of 2..128 columns, a
 * power of two, and d = 2..8; else as -1), 3 = lane form without the minimum
 * corners (kept for comparisons).  The result never depends on the form; this
 * is for tests and tuning sweeps.  SKYCELL_REFINE_FORM=lane|wave|tile|plain in
 * the environment sets it at the first call.
 */
int skycell_set_refine_form(int32_t form);

/*
 * Waves per work item of the wave form for all later calls in the process:
 * 0 = chosen per call (the tuning table's parts column for the call's d, n and
 * grid, else 1), 1..64 = that many.  With p parts, p waves walk the same item's
 * lower cone and each screens every p-th group of its candidates, so a cone
 * that holds most of the input is shared by p waves instead of one.  The
 * result never depends on it.  Returns SKYCELL_E_INVAL outside [0, 64].
 * SKYCELL_WAVE_PARTS in the environment sets it at the first call.
 */
int skycell_set_wave_parts(int32_t parts);

/*
 * Sampling gate of the pivot pre-filter (skycell_compute_with_pivots,
 * skycell_compute_pivoted) for all later calls in the process: 1 (the default)
 * screens a sample first and skips the full pass when the pivots remove fewer
 * than 1 in 100 of its points; 0 always runs the full pass, so that every point
 * of a surviving cell that a pivot dominates is removed.  The skyline never
 * depends on it.  Returns SKYCELL_E_INVAL unless on is 0 or 1.
 */
int skycell_set_pivot_gate(int32_t on);

/*
 * Cell prune of skycell_compute, skycell_compute_u16 and skycell_compute_ws for
 * all later calls in the process (the _static, batched and pivoted forms
 * always use 0).  With form 1, skycell_compute_ws also allocates the tree's
 * scratch (library-owned, kept per device and stream), so this measurement
 * mode is not for callers that must not allocate:
 *   0  (default) Definition 3 by a prefix-OR of the occupancy along each
 *      dimension: a non-empty cell survives iff no non-empty cell has a
 *      smaller column in every dimension;
 *   1  the paper's parallel ShrinkKeyCells (Section V-B, Algorithm 3) run
 *      layer by layer as in Algorithm 1 (layer i has 2^i columns; layer i+1's
 *      leaves are the 2^d children of layer i's key and candidate cells), for
 *      grids of g = 2^rho columns (other grids keep form 0).  Its verdicts
 *      are one-sided (a cell it calls dominated is dominated, but it keeps some
 *      dominated cells: Theorem 2 does not hold in general), so it keeps a
 *      superset of form 0's survivors; the skyline is the same.
 * Returns SKYCELL_E_INVAL unless form is 0 or 1.
 */
int skycell_set_cell_prune(int32_t form);

/*
 * Slab split of the lane refine for all later calls in the process (d <= 8,
 * lane form with minimum corners): the cells with the largest cone-size
 * estimate prod_k (c_k + 1), about 1/256 of the work items, get one work item
 * per slab of their lower cone (the cells with one column of dimension d-1,
 * walked in dimensions 0..d-2), so that the longest cone walks run in
 * parallel on neighbouring lanes instead of holding one lane, and the launch,
 * past the others (Algorithm 1's RefineSkyline; the split changes only how
 * the cone of a cell is divided among lanes).  -1 = on from d = 7 and 2^18
 * points (measured faster there, slower on small calls), 0 = off, 1 = on
 * whenever the form allows it, 2 = as many cells, largest estimate first, as
 * the workspace's n work item slots have room for (for tests).  A split that
 * would need more than those slots is not made.  The result never depends on
 * it.  Returns SKYCELL_E_INVAL unless mode is -1, 0, 1 or 2.
 */
int skycell_set_slab_split(int32_t mode);

/*
 * The tree form's layers on their own, for tests and measurements: the points'
 * occupancy at g = 2^rho (1 <= rho, rho * d <= 26; Equation 1 per layer), then
 * Algorithm 3 for layers 1..rho.  key_out and cand_out (device uint64 bitmaps)
 * receive, for every layer j = 1..rho in turn, one bit per cell of the layer
 * (Morton index: bit b of column k at index bit b*d + k; ceil(2^(j d) / 64)
 * words per layer): key cells, and key plus candidate cells (Theorem 2).
 */
int skycell_shrink_tree(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t rho, int32_t value_bits,
                        uint64_t *key_out, uint64_t *cand_out, void *stream);

/*
 * Byte offsets of the workspace's sub-buffers for (n, d, grid_res) (grid_res 0 =
 * autotuned), for tests and tools that inspect intermediate results of a
 * skycell_compute_ws call.  offsets[0..count) receives, in this order:
 *   0 cell_of  uint32 [n]        Morton index of each point's cell: bit b of column
 *                                c[k] at index bit b*d + k, r = ceil(log2 g) bits
 *   1 rank     uint32 [n]        position of the point among the points of its cell
 *   2 cnt      uint32 [cells]    histogram, cells = 2^(r*d)
 *   3 lc       uint64 [cells/64+1] lower closure of the occupancy, one bit per cell
 *                                (bit x of word x/64: some non-empty cell is <= x)
 *   4 rec      uint64 [cells+1]  per-cell record: bits 0-31 first sorted position,
 *                                32-46 point count (saturated at 0x7FFF), 47-62 mask
 *                                (bit k: the cone one column lower in dimension k
 *                                holds a non-empty cell), 63 surviving non-empty cell
 *   5 keys     uint32 [n*d]      sorted surviving points as order-preserving keys
 *   6 fkeys    uint64 [n*ceil(d/8)]  7-bit screening columns, one byte per dimension
 *   7 sidx     int32  [n]        original index of each sorted point
 *   8 items, 9 flag, 10 block sums, 11 counters, 12 total size (past the
 *   counters: a bitmap of surviving cells, for n >= 2^20 the staging rows of
 *   the two-pass scatter, and for d <= 8 one walk-record word per cell: the
 *   lower-neighbour mask and the cell's minimum screening column per
 *   dimension, read by the lane form of the refine).
 * count must be >= 13.  Returns SKYCELL_OK or an argument error.
 */
int skycell_workspace_layout(int64_t n, int32_t d, int32_t grid_res, int32_t dtype,
                             size_t *offsets, int32_t count);

/*
 * Phase timing.  After skycell_profile_enable(1), every later call on the
 * calling thread records hipEvents on its stream between the phases of the
 * path.  skycell_profile_read waits for the last recorded event and writes the
 * milliseconds of the last profiled call, phase by phase, in this order:
 *   0 init + quantise/histogram (Equation 1)   1 cell prune (Definition 3)
 *   2 cell scan (offsets, work items)          3 scatter of surviving points
 *   4 refine (lower-cone point domination)     5 ordered output
 * count must be >= SKYCELL_NUM_PHASES.  Disabling frees the events.
 */
#define SKYCELL_NUM_PHASES 6
int skycell_profile_enable(int32_t on);
int skycell_profile_read(float *ms, int32_t count);

/*
 * Batched skylines: many independent instances of uneven n and d computed by
 * one hipGraphLaunch.  The plan lays out every instance's workspace in one
 * allocation; at the first run (and again when a run passes other buffers) it
 * captures the single-instance path of every instance into one graph, spread
 * over parallel branches, largest instances first.  Every instance's result
 * equals skycell_compute on its own points.
 *
 *   num_inst   number of instances, >= 1.
 *   n, d       host arrays [num_inst]: points and attributes of each instance
 *              (0 <= n < 2^31, total points below 2^31, 1 <= d <= 16).
 *   dtype      SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16 (value_bits as in
 *              skycell_compute_u16; ignored for F32).
 *   grid_res   host array [num_inst] of cells per dimension (0 entries, or a
 *              NULL array, let the autotuner choose per instance); each grid's
 *              index space is limited to 32 cells per point (at least 2^16,
 *              at most 2^24 cells).
 *   plan       receives an opaque handle owning the device workspace and the
 *              graph.  Creating a plan allocates device memory; it is not
 *              capture-safe.
 *
 * Buffers of a run (device memory, caller-owned):
 *   points     instance b occupies elements [P_b, P_{b+1}) as an SoA block
 *              [d_b][n_b] (attribute k of point i at P_b + k*n_b + i), with
 *              P_b = sum_{a<b} n_a * d_a (skycell_batched_offsets gives P).
 *   out_idx    int32 [sum n]: instance b's skyline indices (local, 0..n_b-1,
 *              ascending) start at O_b = sum_{a<b} n_a.
 *   out_count  int32 [num_inst]: skyline size of each instance, or
 *              SKYCELL_E_NAN if the instance holds a NaN.
 * A run is one hipGraphLaunch on `stream`; capturing (first run, or new
 * buffers) costs host time proportional to the number of instances, so pass
 * the same buffers to replay.  Runs of one plan must not overlap in time (they
 * share the plan's workspace).
 */
typedef struct skycell_plan *skycell_plan_t;

int skycell_batched_plan_create(int32_t num_inst, const int64_t *n, const int32_t *d, int32_t dtype,
                                int32_t value_bits, const int32_t *grid_res, skycell_plan_t *plan);

/* Host arrays [num_inst + 1] of element offsets P_b and output offsets O_b, and
 * [num_inst] of the grid chosen per instance; any pointer may be NULL. */
int skycell_batched_offsets(skycell_plan_t plan, int64_t *points_off, int64_t *out_off,
                            int32_t *grid_res);

int skycell_batched_run(skycell_plan_t plan, const void *points, int32_t *out_idx,
                        int32_t *out_count, void *stream);

/* Waits for the device, then frees the plan's memory and graph. */
int skycell_plan_destroy(skycell_plan_t plan);

/*
 * ------------------------------------------------------------------------
 * Incremental maintenance under inserts and deletes.
 *
 * The paper holds (Section I; Section VII-B3, dynamic scenarios) that SkyCell
 * needs no pre-computation, so updates do not invalidate anything it keeps.
 * A skycell_dyn_t keeps a point set in library-owned device memory with each
 * point's skyline flag (Definition 2 over the live points) and updates it per
 * batch by recomputing only the points the batch can change:
 *   insert B: sky(P + B) = sky(S + B) with S the current skyline (a dominated
 *             point stays dominated when points are added);
 *   delete D: sky(P - D) = sky((S - D) + R), R = the live non-skyline points
 *             that some deleted skyline point is <= in every dimension.
 * The recompute is the whole single-instance path on the gathered points.
 * Ids are insertion positions 0, 1, 2, ... and are never reused.  Each update
 * synchronises the stream (it reads candidate counts back) and returns once
 * the flags are final.  Calls on one handle are serialised by the library.
 */
typedef struct skycell_dyn *skycell_dyn_t;

/* capacity: ids available over the handle's life (1 <= capacity < 2^31).
 * dtype SKYCELL_DTYPE_F32 or SKYCELL_DTYPE_U16 (value_bits as for
 * skycell_compute_u16; ignored for F32).  Allocates capacity * (2 d esize + 11)
 * bytes on the current device; the recompute's workspace grows on demand. */
int skycell_dyn_create(int32_t d, int32_t dtype, int64_t capacity, int32_t value_bits, skycell_dyn_t *out);

/* Append m points (device SoA [d][m], the handle's dtype) as ids first_id ..
 * first_id + m - 1 (*first_id may be NULL).  SKYCELL_E_NOMEM when the capacity
 * would be exceeded, SKYCELL_E_NAN when the batch holds a NaN; in both cases
 * nothing is inserted. */
int skycell_dyn_insert(skycell_dyn_t h, const void *points, int64_t m, int64_t *first_id, void *stream);

/* Delete the ids in ids[0..m) (device int32).  Deleted and repeated ids are
 * ignored; an id outside [0, ids used) makes it return SKYCELL_E_RANGE after
 * the valid ids of the batch were deleted and the skyline updated. */
int skycell_dyn_delete(skycell_dyn_t h, const int32_t *ids, int64_t m, void *stream);

/* The current skyline as ascending ids (device int32, capacity >= ids used)
 * and its size (device int32), enqueued on the stream. */
int skycell_dyn_skyline(skycell_dyn_t h, int32_t *out_idx, int32_t *out_count, void *stream);

/* Ids handed out so far, and how many points the last update recomputed. */
int skycell_dyn_size(skycell_dyn_t h, int64_t *ids_used, int64_t *last_candidates);

/* Waits for the device, then frees the handle's memory. */
int skycell_dyn_destroy(skycell_dyn_t h);

/*
 * ------------------------------------------------------------------------
 * Quadrant (dynamic-origin) skyline queries, Section VII-B3.
 *
 * A query point o is taken as the new origin and only the points of its
 * top-right quadrant Q(o) = { p : p[k] >= o[k] for every k } (closed, compared
 * exactly; -0.0 = +0.0) take part: the answer to the query is the skyline of
 * Q(o) (Definitions 1-2), as ascending indices into the data set.  Many
 * queries on one resident data set run as the instances of one batched plan
 * (skycell_batched_*): the create call measures |Q(o)| for every query and
 * lays the plan out; each run gathers the quadrants, launches the plan's graph
 * once, and writes every query's skyline.
 */
typedef struct skycell_quad *skycell_quad_t;

/* points: device SoA [d][n] (dtype F32 or U16; value_bits as for
 * skycell_compute_u16).  origins: device SoA [d][nq] of the same dtype
 * (1 <= nq <= 4,194,240).  Counts the quadrants (synchronises the stream) and
 * allocates the plan; the quadrants together must hold fewer than 2^31 points
 * (else SKYCELL_E_RANGE).  A NaN origin gives SKYCELL_E_NAN. */
int skycell_quadrant_create(const void *points, int32_t dtype, int64_t n, int32_t d, int32_t value_bits,
                            const void *origins, int32_t nq, skycell_quad_t *out, void *stream);

/* out_off[0..nq]: query q's skyline goes to out_idx[out_off[q] ..] (room for
 * |Q(o_q)| indices); out_off[nq] is the capacity out_idx needs. */
int skycell_quadrant_offsets(skycell_quad_t h, int64_t *out_off);

/* Answer every query for the same points and origins the handle was created
 * with: out_idx (device int32, capacity out_off[nq]) receives at out_off[q]
 * the ascending skyline of query q, out_count (device int32 [nq]) its size (or
 * SKYCELL_E_NAN when Q(o_q) holds a NaN).  The first run captures the graph. */
int skycell_quadrant_run(skycell_quad_t h, const void *points, const void *origins, int32_t *out_idx,
                         int32_t *out_count, void *stream);

/* Waits for the device, then frees the handle and its plan. */
int skycell_quadrant_destroy(skycell_quad_t h);

/*
 * ------------------------------------------------------------------------
 * Learned pivot proposer and pivot pre-filter.
 *
 * Not part of the paper's method: a small network scores points by how likely
 * they are to be skyline points, and the best-scoring points serve as pivots.
 * A pivot v removes every point q of a surviving cell that it dominates
 * (Definition 1) before the counting sort, so q is neither refined nor used as
 * a candidate.  The pass is gated: points i = j * (n / m), j < m = min(n,
 * 16384) (integer division) are screened first, and the pass runs only when
 * at least 1 in 100 of the sampled points of surviving cells is dominated by
 * a pivot (or none was sampled); otherwise no point is removed.  The skyline is unchanged (dominance is transitive, so every
 * remaining point keeps an undominated dominator in its lower cone): the
 * result of every pivoted call equals skycell_compute's, whatever the pivots.
 *
 * Network: features f = (x[0..d), frac(x[k] * g) for k < d) of a point x, with
 * the binary32 product x[k] * g and frac(t) = t - floor(t) (its position inside
 * its column of Equation 1, g = the network's grid_res); then
 *   h1 = relu(W1 f + b1), h2 = relu(W2 h1 + b2), logit = w3 . h2 + b3,
 * 2d -> 64 -> 64 -> 1.  Weights are kept in float32 (master copy, Adam state)
 * and used as bfloat16 (round to nearest even); features and hidden
 * activations are rounded to bfloat16 before each matrix product, which runs
 * on the matrix cores with float32 accumulation.  Flat float32 parameter
 * order: W1 [64][2d] (output-unit major), b1 [64], W2 [64][64], b2 [64],
 * w3 [64], b3 — 128 d + 4289 values.
 *
 * Training minimises the mean binary cross-entropy of sigmoid(logit) against
 * skyline labels (1 = skyline point) with Adam (beta1 0.9, beta2 0.999,
 * epsilon 1e-8, bias-corrected).  Gradients pass straight through the
 * bfloat16 roundings; the back-propagated pre-activation gradients are rounded
 * to bfloat16 where they enter a matrix product.
 *
 * Points here are SoA blocks with a leading dimension: attribute k of point i
 * at points[k * ld + i], ld >= n (ld = n for a whole array; a larger ld with an
 * offset base pointer selects a mini-batch of a bigger array).
 * Handles are bound to the device current at creation; every call on a handle
 * must run with that device current.  Calls on one handle must not overlap.
 * ------------------------------------------------------------------------
 */
#define SKYCELL_MLP_HIDDEN 64
#define SKYCELL_MAX_PIVOTS 4096

typedef struct skycell_mlp *skycell_mlp_t;

/* Number of float32 parameters for d attributes (128 d + 4289). */
int skycell_mlp_num_params(int32_t d, int64_t *count);

/* New network for d attributes (1..16) and feature grid grid_res (>= 1):
 * Glorot-uniform weights drawn from a counter-based generator (SplitMix64 of
 * seed + parameter index), zero biases, zero Adam state.  Allocates device
 * memory and synchronises the device. */
int skycell_mlp_create(int32_t d, int32_t grid_res, uint64_t seed, skycell_mlp_t *mlp);
int skycell_mlp_destroy(skycell_mlp_t mlp);

/* Host float32 [count] parameters in the flat order above; count must equal
 * skycell_mlp_num_params.  set also clears the Adam state and step count.
 * Both synchronise the device. */
int skycell_mlp_set_params(skycell_mlp_t mlp, const float *params, int64_t count);
int skycell_mlp_get_params(skycell_mlp_t mlp, float *params, int64_t count);

/* Host float32 [count]: the mean gradient of the last skycell_mlp_backward
 * (get), or a gradient for the next skycell_mlp_adam_step (set).  Both
 * synchronise the device. */
int skycell_mlp_get_grads(skycell_mlp_t mlp, float *grads, int64_t count);
int skycell_mlp_set_grads(skycell_mlp_t mlp, const float *grads, int64_t count);

/* Logits of n points (device SoA with leading dimension ld) into device
 * float32 logits [n]. */
int skycell_mlp_score(skycell_mlp_t mlp, const float *points, int64_t ld, int64_t n, float *logits,
                      void *stream);

/* Mean loss and gradient over n points with device uint8 labels [n] (nonzero =
 * skyline point); loss_out (device float32 [1]) may be NULL.  The gradient
 * stays on the device for skycell_mlp_adam_step. */
int skycell_mlp_backward(skycell_mlp_t mlp, const float *points, int64_t ld, const uint8_t *labels,
                         int64_t n, float *loss_out, void *stream);

/* One Adam step with learning rate lr on the current gradient. */
int skycell_mlp_adam_step(skycell_mlp_t mlp, float lr, void *stream);

/* skycell_mlp_backward followed by skycell_mlp_adam_step. */
int skycell_mlp_train_step(skycell_mlp_t mlp, const float *points, int64_t ld, const uint8_t *labels,
                           int64_t n, float lr, float *loss_out, void *stream);

/* Binary file: "SKYMLP01", int32 d, grid_res, step, count, then float32
 * parameters, first and second Adam moments (count each), little-endian. */
int skycell_mlp_save(skycell_mlp_t mlp, const char *path);
int skycell_mlp_load(const char *path, skycell_mlp_t *mlp);

/* Training labels from a skyline result: labels[i] = 1 iff i is among
 * idx[0 .. *count) (device pointers; a negative *count gives all zeros). */
int skycell_skyline_labels(const int32_t *idx, const int32_t *count, int64_t n, uint8_t *labels,
                           void *stream);

/* Indices of the min(k, n) largest scores (device float32 [n]), largest first,
 * equal scores (-0.0 == +0.0) by ascending index, into device int32 out_idx;
 * 1 <= k <= SKYCELL_MAX_PIVOTS.  NaN scores take the place their bit pattern's
 * order key gives them. */
int skycell_topk(const float *scores, int64_t n, int32_t k, int32_t *out_idx, void *stream);

/* skycell_compute (binary32) with the pre-filter by k caller-chosen pivots
 * (device int32 pivot_idx [k], 0 <= k <= SKYCELL_MAX_PIVOTS).  A pivot index
 * outside [0, n) makes *out_count = SKYCELL_E_RANGE.  stats as in
 * skycell_compute_ws (may be NULL). */
int skycell_compute_with_pivots(const float *points, int64_t n, int32_t d, int32_t grid_res,
                                const int32_t *pivot_idx, int32_t k, int32_t *out_idx, int32_t *out_count,
                                uint64_t *stats, void *stream);

/* skycell_compute (binary32) with the k best-scoring points of mlp as pivots
 * (mlp's d must equal d).  Output identical to skycell_compute. */
int skycell_compute_pivoted(const float *points, int64_t n, int32_t d, int32_t grid_res, skycell_mlp_t mlp,
                            int32_t k, int32_t *out_idx, int32_t *out_count, uint64_t *stats, void *stream);

/* Text for the last nonzero return of the calling thread ("" if none). */
const char *skycell_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SKYCELL_H */
