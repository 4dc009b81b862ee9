"""MI355X (gfx950) exact skyline following SkyCell (arXiv 2107.09993).

Thin Python binding over the C ABI of ``libskycell.so`` (declared in
``include/skycell.h``).  It only marshals arguments: PyTorch provides device
memory and the stream, every step of the skyline runs in the library's HIP
kernels.  There is no CPU fallback; if the library is missing, calls raise.

    import torch, paper_2107_09993_amd as sky
    x = torch.rand(1_000_000, 8, device="cuda")
    idx = sky.compute(x)          # ascending int32 indices of the skyline points
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libskycell.so")

OK = 0
E_INVAL = -1
E_RANGE = -2
E_NOMEM = -3
E_HIP = -4
E_NODEV = -5
E_NAN = -6
MAX_D = 16
MAX_CELLS = 1 << 26
DTYPE_F32 = 0
DTYPE_U16 = 1
NUM_STATS = 9
STAT_NAMES = ("nonempty_cells", "surviving_cells", "survivor_points", "items", "cell_visits",
              "pair_tests", "skyline", "grid_res", "pivot_removed")
STATIC_SCRATCH_BYTES = 64 << 20
MLP_HIDDEN = 64
MAX_PIVOTS = 4096

_lib = None


class SkycellError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("skycell error %d: %s" % (code, msg))
        self.code = code


def lib():
    """The loaded ctypes library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libskycell.so is not built (run: python -m paper_2107_09993_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    i64, i32, p, sz = ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t
    L.skycell_compute.argtypes = [p, i64, i32, i32, p, p, p]
    L.skycell_compute_u16.argtypes = [p, i64, i32, i32, i32, p, p, p]
    L.skycell_workspace_bytes.argtypes = [i64, i32, i32, i32, ctypes.POINTER(sz)]
    L.skycell_compute_ws.argtypes = [p, i32, i64, i32, i32, i32, p, p, p, sz, p, p]
    L.skycell_compute_static.argtypes = [p, i32, i64, i32, i32, i32, p, p, p, p]
    L.skycell_choose_grid.argtypes = [i64, i32, i32, ctypes.POINTER(i32)]
    L.skycell_input_class.argtypes = [p, i32, i64, i32, ctypes.POINTER(i32), p]
    L.skycell_choose_config.argtypes = [i64, i32, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32),
                                        ctypes.POINTER(i32)]
    L.skycell_load_tuning.argtypes = [ctypes.c_char_p]
    L.skycell_set_refine_form.argtypes = [i32]
    L.skycell_set_slab_split.argtypes = [i32]
    L.skycell_set_wave_parts.argtypes = [i32]
    L.skycell_set_pivot_gate.argtypes = [i32]
    L.skycell_set_cell_prune.argtypes = [i32]
    L.skycell_compute_layered.argtypes = [p, i32, i64, i32, i32, i32, p, p, p, p]
    L.skycell_shrink_tree.argtypes = [p, i32, i64, i32, i32, i32, p, p, p]
    L.skycell_workspace_layout.argtypes = [i64, i32, i32, i32, ctypes.POINTER(sz), i32]
    L.skycell_profile_enable.argtypes = [i32]
    L.skycell_profile_read.argtypes = [ctypes.POINTER(ctypes.c_float), i32]
    L.skycell_batched_plan_create.argtypes = [i32, p, p, i32, i32, p, ctypes.POINTER(p)]
    L.skycell_batched_offsets.argtypes = [p, p, p, p]
    L.skycell_batched_run.argtypes = [p, p, p, p, p]
    L.skycell_plan_destroy.argtypes = [p]
    L.skycell_mlp_num_params.argtypes = [i32, ctypes.POINTER(i64)]
    L.skycell_mlp_create.argtypes = [i32, i32, ctypes.c_uint64, ctypes.POINTER(p)]
    L.skycell_mlp_destroy.argtypes = [p]
    L.skycell_mlp_set_params.argtypes = [p, p, i64]
    L.skycell_mlp_get_params.argtypes = [p, p, i64]
    L.skycell_mlp_get_grads.argtypes = [p, p, i64]
    L.skycell_mlp_set_grads.argtypes = [p, p, i64]
    L.skycell_mlp_score.argtypes = [p, p, i64, i64, p, p]
    L.skycell_mlp_backward.argtypes = [p, p, i64, p, i64, p, p]
    L.skycell_mlp_adam_step.argtypes = [p, ctypes.c_float, p]
    L.skycell_mlp_train_step.argtypes = [p, p, i64, p, i64, ctypes.c_float, p, p]
    L.skycell_mlp_save.argtypes = [p, ctypes.c_char_p]
    L.skycell_mlp_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(p)]
    L.skycell_skyline_labels.argtypes = [p, p, i64, p, p]
    L.skycell_topk.argtypes = [p, i64, i32, p, p]
    L.skycell_compute_with_pivots.argtypes = [p, i64, i32, i32, p, i32, p, p, p, p]
    L.skycell_compute_pivoted.argtypes = [p, i64, i32, i32, p, i32, p, p, p, p]
    L.skycell_dyn_create.argtypes = [i32, i32, i64, i32, ctypes.POINTER(p)]
    L.skycell_dyn_insert.argtypes = [p, p, i64, ctypes.POINTER(i64), p]
    L.skycell_dyn_delete.argtypes = [p, p, i64, p]
    L.skycell_dyn_skyline.argtypes = [p, p, p, p]
    L.skycell_dyn_size.argtypes = [p, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.skycell_dyn_destroy.argtypes = [p]
    L.skycell_quadrant_create.argtypes = [p, i32, i64, i32, i32, p, i32, ctypes.POINTER(p), p]
    L.skycell_quadrant_offsets.argtypes = [p, p]
    L.skycell_quadrant_run.argtypes = [p, p, p, p, p, p]
    L.skycell_quadrant_destroy.argtypes = [p]
    L.skycell_last_error.argtypes = []
    L.skycell_last_error.restype = ctypes.c_char_p
    for name in ("skycell_compute", "skycell_compute_u16", "skycell_workspace_bytes",
                 "skycell_compute_ws", "skycell_compute_static", "skycell_choose_grid", "skycell_load_tuning", "skycell_set_refine_form",
                 "skycell_input_class", "skycell_choose_config",
                 "skycell_set_wave_parts", "skycell_set_pivot_gate", "skycell_set_cell_prune",
                 "skycell_set_slab_split",
                 "skycell_shrink_tree", "skycell_compute_layered",
                 "skycell_workspace_layout", "skycell_profile_enable", "skycell_profile_read",
                 "skycell_batched_plan_create", "skycell_batched_offsets", "skycell_batched_run",
                 "skycell_plan_destroy", "skycell_mlp_num_params", "skycell_mlp_create",
                 "skycell_mlp_destroy", "skycell_mlp_set_params", "skycell_mlp_get_params",
                 "skycell_mlp_get_grads", "skycell_mlp_set_grads", "skycell_mlp_score",
                 "skycell_mlp_backward", "skycell_mlp_adam_step", "skycell_mlp_train_step",
                 "skycell_mlp_save", "skycell_mlp_load", "skycell_skyline_labels", "skycell_topk",
                 "skycell_compute_with_pivots", "skycell_compute_pivoted",
                 "skycell_dyn_create", "skycell_dyn_insert", "skycell_dyn_delete", "skycell_dyn_skyline",
                 "skycell_dyn_size", "skycell_dyn_destroy", "skycell_quadrant_create",
                 "skycell_quadrant_offsets", "skycell_quadrant_run", "skycell_quadrant_destroy"):
        getattr(L, name).restype = i32
    _lib = L
    table = os.path.join(HERE, "tuning", "mi355x.txt")
    if os.path.exists(table) and os.environ.get("SKYCELL_NO_TUNING") is None:
        L.skycell_load_tuning(table.encode())
    return L


def _check(rc):
    if rc != OK:
        raise SkycellError(rc, lib().skycell_last_error().decode())


def last_error():
    return lib().skycell_last_error().decode()


def workspace_bytes(n, d, grid_res=0, dtype=DTYPE_F32):
    out = ctypes.c_size_t(0)
    _check(lib().skycell_workspace_bytes(int(n), int(d), int(grid_res), int(dtype), ctypes.byref(out)))
    return out.value


def choose_grid(n, d, dtype=DTYPE_F32):
    g = ctypes.c_int32(0)
    _check(lib().skycell_choose_grid(int(n), int(d), int(dtype), ctypes.byref(g)))
    return g.value


CLASS_INDEPENDENT, CLASS_CORRELATED, CLASS_ANTICORRELATED = 0, 1, 2
CLASS_NAMES = ("independent", "correlated", "anticorrelated")


def input_class(points_soa, stream=None):
    """Input class (CLASS_*) of a contiguous [d, n] CUDA tensor, float32 or
    uint16 (skycell_input_class; waits for the stream)."""
    import torch
    if not points_soa.is_cuda or not points_soa.is_contiguous() or points_soa.dim() != 2:
        raise ValueError("points must be a contiguous [d, n] CUDA tensor")
    d, n = points_soa.shape
    st = stream if stream is not None else torch.cuda.current_stream(points_soa.device).cuda_stream
    c = ctypes.c_int32(-1)
    _check(lib().skycell_input_class(ctypes.c_void_p(points_soa.data_ptr()), _dtype_code(points_soa), int(n),
                                     int(d), ctypes.byref(c), ctypes.c_void_p(st)))
    return c.value


def choose_config(n, d, dtype=DTYPE_F32, cls=-1):
    """(grid, refine form name, waves per item) a grid_res = 0 call uses for an
    input of class cls (-1: not known), from the tuning table."""
    g, f, p = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    _check(lib().skycell_choose_config(int(n), int(d), int(dtype), int(cls), ctypes.byref(g), ctypes.byref(f),
                                       ctypes.byref(p)))
    return g.value, ("lane", "wave")[f.value], p.value


NUM_PHASES = 6
PHASE_NAMES = ("quantize_hist", "cell_prune", "cell_scan", "scatter", "refine", "output")


def profile_enable(on=True):
    _check(lib().skycell_profile_enable(1 if on else 0))


def profile_read():
    """Milliseconds per phase of the last profiled call on this thread (waits for it)."""
    ms = (ctypes.c_float * NUM_PHASES)()
    _check(lib().skycell_profile_read(ms, NUM_PHASES))
    return dict(zip(PHASE_NAMES, (float(v) for v in ms)))


def workspace_layout(n, d, grid_res=0, dtype=DTYPE_F32):
    offs = (ctypes.c_size_t * 13)()
    _check(lib().skycell_workspace_layout(int(n), int(d), int(grid_res), int(dtype), offs, 13))
    return list(offs)


REFINE_FORMS = {"auto": -1, "lane": 0, "wave": 1, "tile": 2, "plain": 3}


def set_refine_form(form):
    """Refine form for later calls: "auto" (per call), "lane", "wave", "tile" or
    "plain" (the lane form without the minimum-corner screen)."""
    _check(lib().skycell_set_refine_form(REFINE_FORMS[form]))


def set_wave_parts(parts):
    """Waves per work item of the wave-form refine for later calls (0 = per call)."""
    _check(lib().skycell_set_wave_parts(int(parts)))


def set_pivot_gate(on):
    """Sampling gate of the pivot pre-filter for later calls: True (default)
    skips the full pass when a sample shows almost nothing to remove; False
    always screens every point of a surviving cell against the pivots."""
    _check(lib().skycell_set_pivot_gate(1 if on else 0))


SLAB_SPLIT_MODES = {"auto": -1, "off": 0, "on": 1, "all": 2}


def set_slab_split(mode):
    """Slab split of the lane refine's longest cone walks for later calls:
    "auto" (from d = 7 and 2^18 points), "off", "on" or "all" (as many cells
    as the item array has room for; for tests)."""
    _check(lib().skycell_set_slab_split(SLAB_SPLIT_MODES[mode]))


CELL_PRUNE_FORMS = {"prefix_or": 0, "tree": 1}


def set_cell_prune(form):
    """Cell prune of compute() for later calls: "prefix_or" (Definition 3, the
    default) or "tree" (the paper's Algorithm 3 per layer; g = 2^rho only)."""
    _check(lib().skycell_set_cell_prune(CELL_PRUNE_FORMS[form]))


def shrink_tree_layers(points_soa, rho, value_bits=10):
    """Algorithm 3 layer by layer on a contiguous [d, n] device tensor: a list,
    per layer 1..rho, of (key_bits, cand_bits) numpy uint64 bitmaps over the
    layer's Morton-numbered cells."""
    import numpy as np
    import torch
    d, n = (int(v) for v in points_soa.shape)
    words = [((1 << (j * d)) + 63) // 64 for j in range(1, rho + 1)]
    total = max(sum(words), 1)
    key = torch.zeros(total, dtype=torch.int64, device=points_soa.device)
    cand = torch.zeros(total, dtype=torch.int64, device=points_soa.device)
    st = ctypes.c_void_p(torch.cuda.current_stream(points_soa.device).cuda_stream)
    _check(lib().skycell_shrink_tree(ctypes.c_void_p(points_soa.data_ptr()), _dtype_code(points_soa), n, d,
                                     int(rho), int(value_bits), ctypes.c_void_p(key.data_ptr()),
                                     ctypes.c_void_p(cand.data_ptr()), st))
    k = key.cpu().numpy().view(np.uint64)
    c = cand.cpu().numpy().view(np.uint64)
    out, off = [], 0
    for w in words:
        out.append((k[off:off + w], c[off:off + w]))
        off += w
    return out


def load_tuning(path):
    _check(lib().skycell_load_tuning(path.encode() if path else None))


def _dtype_code(t):
    import torch
    if t.dtype == torch.float32:
        return DTYPE_F32
    if t.dtype == torch.uint16:
        return DTYPE_U16
    raise TypeError("points must be float32 or uint16, got %s" % t.dtype)


def to_soa(points):
    """[n, d] tensor -> contiguous [d, n] (structure of arrays) on the same device."""
    return points.t().contiguous()


class Skyline:
    """Reusable buffers for repeated skyline calls on one shape (device memory from torch).

    ``run(points_soa)`` enqueues the whole path on the current stream and returns the
    device tensors (out_idx, out_count) without synchronising.
    """

    def __init__(self, n, d, dtype="f32", grid_res=0, value_bits=10, device="cuda", stats=False):
        import torch
        self.n, self.d = int(n), int(d)
        self.dtype = DTYPE_F32 if dtype in ("f32", DTYPE_F32) else DTYPE_U16
        self.value_bits = int(value_bits) if self.dtype == DTYPE_U16 else 16
        self.grid_res = grid_res if grid_res else choose_grid(self.n, self.d, self.dtype)
        self.device = torch.device(device)
        self.ws_bytes = workspace_bytes(self.n, self.d, self.grid_res, self.dtype)
        self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        self.out_idx = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.device)
        self.out_count = torch.empty(1, dtype=torch.int32, device=self.device)
        self.stats = torch.zeros(NUM_STATS, dtype=torch.int64, device=self.device) if stats else None

    def run(self, points_soa, stream=None):
        import torch
        if points_soa.device != self.device or not points_soa.is_contiguous():
            raise ValueError("points must be a contiguous [d, n] tensor on %s" % self.device)
        if tuple(points_soa.shape) != (self.d, self.n):
            raise ValueError("points must have shape (%d, %d), got %s" % (self.d, self.n, tuple(points_soa.shape)))
        if _dtype_code(points_soa) != self.dtype:
            raise TypeError("dtype mismatch")
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        rc = lib().skycell_compute_ws(
            ctypes.c_void_p(points_soa.data_ptr()), self.dtype, self.n, self.d, self.grid_res,
            self.value_bits, ctypes.c_void_p(self.out_idx.data_ptr()),
            ctypes.c_void_p(self.out_count.data_ptr()), ctypes.c_void_p(self.workspace.data_ptr()),
            self.ws_bytes, ctypes.c_void_p(self.stats.data_ptr()) if self.stats is not None else None,
            ctypes.c_void_p(st))
        _check(rc)
        return self.out_idx, self.out_count

    def result(self):
        """Synchronise on the count and return the skyline indices (int32 tensor)."""
        c = int(self.out_count.item())
        if c < 0:
            raise SkycellError(c, "device reported %s" % ("NaN in input" if c == E_NAN else "error"))
        return self.out_idx[:c]

    def stats_dict(self):
        if self.stats is None:
            return {}
        return dict(zip(STAT_NAMES, (int(v) for v in self.stats.cpu().tolist())))


def compute(points, grid_res=0, layout="nd", value_bits=10, return_stats=False):
    """Exact skyline of a CUDA tensor of points (float32 or uint16).

    layout "nd": points is [n, d] (transposed to SoA first); "dn": points is [d, n].
    Returns ascending int32 indices (a CUDA tensor); with return_stats also a dict
    of the library's counters.
    """
    if not points.is_cuda:
        raise ValueError("points must be a CUDA (HIP) tensor")
    soa = to_soa(points) if layout == "nd" else points.contiguous()
    d, n = soa.shape
    sk = Skyline(n, d, dtype=_dtype_code(soa), grid_res=grid_res, value_bits=value_bits,
                 device=soa.device, stats=return_stats)
    sk.run(soa)
    out = sk.result().clone()
    if return_stats:
        return out, sk.stats_dict()
    return out


def compute_layered(points_soa, rho, value_bits=10, return_stats=False):
    """Exact skyline of a contiguous [d, n] tensor with two grid layers: the
    dense base grid of 2^(rho-1) columns and an exact Definition 3 prune at
    2^rho columns kept as occupancy bits (skycell_compute_layered)."""
    import torch
    if not points_soa.is_contiguous() or points_soa.dim() != 2:
        raise ValueError("points must be a contiguous [d, n] tensor")
    d, n = (int(v) for v in points_soa.shape)
    dev = points_soa.device
    out_idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    out_count = torch.empty(1, dtype=torch.int32, device=dev)
    stats = torch.zeros(NUM_STATS, dtype=torch.int64, device=dev) if return_stats else None
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    _check(lib().skycell_compute_layered(ctypes.c_void_p(points_soa.data_ptr()), _dtype_code(points_soa), n, d,
                                         int(rho), int(value_bits), ctypes.c_void_p(out_idx.data_ptr()),
                                         ctypes.c_void_p(out_count.data_ptr()),
                                         ctypes.c_void_p(stats.data_ptr()) if stats is not None else None, st))
    c = int(out_count.item())
    if c < 0:
        raise SkycellError(c, "device reported %s" % ("NaN in input" if c == E_NAN else "error"))
    out = out_idx[:c].clone()
    if return_stats:
        return out, dict(zip(STAT_NAMES, (int(v) for v in stats.cpu().tolist())))
    return out


def compute_static(points_soa, grid_res=0, value_bits=10, out_idx=None, out_count=None, stats=None,
                   stream=None):
    """Skyline of a contiguous [d, n] tensor with the library's fixed scratch
    array (skycell_compute_static: no device allocation inside the library).
    out_idx (int32 [n]) and out_count (int32 [1]) may be passed in so that the
    call allocates nothing at all; returns (out_idx, out_count) unsynchronised."""
    import torch
    if not points_soa.is_contiguous() or points_soa.dim() != 2:
        raise ValueError("points must be a contiguous [d, n] tensor")
    d, n = points_soa.shape
    dev = points_soa.device
    if out_idx is None:
        out_idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    if out_count is None:
        out_count = torch.empty(1, dtype=torch.int32, device=dev)
    _check(lib().skycell_compute_static(_ptr(points_soa), _dtype_code(points_soa), n, d, int(grid_res),
                                        int(value_bits), _ptr(out_idx), _ptr(out_count), _ptr(stats),
                                        _stream(dev, stream)))
    return out_idx, out_count


class Dynamic:
    """A point set kept on the device with its skyline, updated per batch of
    inserts and deletes (skycell_dyn_*).  Ids are insertion positions."""

    def __init__(self, d, capacity, dtype="f32", value_bits=10, device="cuda"):
        import torch
        self.d = int(d)
        self.capacity = int(capacity)
        self.dtype = DTYPE_F32 if dtype in ("f32", DTYPE_F32) else DTYPE_U16
        self.device = torch.device(device)
        handle = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib().skycell_dyn_create(self.d, self.dtype, self.capacity, int(value_bits),
                                            ctypes.byref(handle)))
        self.handle = handle
        self.out_idx = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        self.out_count = torch.empty(1, dtype=torch.int32, device=self.device)

    def _stream(self):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def insert(self, points_soa):
        """Append a contiguous [d, m] device tensor; returns the first new id."""
        if tuple(points_soa.shape[:1]) != (self.d,) or not points_soa.is_contiguous():
            raise ValueError("points must be a contiguous [%d, m] tensor" % self.d)
        if _dtype_code(points_soa) != self.dtype:
            raise TypeError("dtype mismatch")
        first = ctypes.c_int64(0)
        _check(lib().skycell_dyn_insert(self.handle, ctypes.c_void_p(points_soa.data_ptr()),
                                        int(points_soa.shape[1]), ctypes.byref(first), self._stream()))
        return first.value

    def delete(self, ids):
        """Delete the ids of a device int32 tensor."""
        import torch
        ids = ids.to(device=self.device, dtype=torch.int32).contiguous()
        _check(lib().skycell_dyn_delete(self.handle, ctypes.c_void_p(ids.data_ptr()), int(ids.numel()),
                                        self._stream()))

    def skyline(self):
        """Current skyline: ascending ids (int32 device tensor)."""
        _check(lib().skycell_dyn_skyline(self.handle, ctypes.c_void_p(self.out_idx.data_ptr()),
                                         ctypes.c_void_p(self.out_count.data_ptr()), self._stream()))
        c = int(self.out_count.item())
        return self.out_idx[:c].clone()

    def size(self):
        """(ids used, points recomputed by the last update)."""
        used, last = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(lib().skycell_dyn_size(self.handle, ctypes.byref(used), ctypes.byref(last)))
        return used.value, last.value

    def close(self):
        if self.handle:
            _check(lib().skycell_dyn_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class QuadrantQueries:
    """Quadrant skyline queries (Section VII-B3) on one resident data set: query
    q answers with the skyline of the points p >= origins[q] (every dimension).

    points_soa: contiguous [d, n] device tensor; origins_soa: contiguous [d, nq]
    device tensor of the same dtype.  run() enqueues every query (one graph
    launch) and returns (out_idx, out_count) device tensors; answers() splits
    them into per-query numpy arrays of ascending indices.
    """

    def __init__(self, points_soa, origins_soa, value_bits=10):
        import numpy as np
        import torch
        if points_soa.dim() != 2 or origins_soa.dim() != 2 or not points_soa.is_contiguous() \
                or not origins_soa.is_contiguous():
            raise ValueError("points and origins must be contiguous [d, n] and [d, nq] tensors")
        self.d, self.n = (int(v) for v in points_soa.shape)
        if int(origins_soa.shape[0]) != self.d:
            raise ValueError("origins must have %d rows" % self.d)
        self.nq = int(origins_soa.shape[1])
        self.dtype = _dtype_code(points_soa)
        if _dtype_code(origins_soa) != self.dtype:
            raise TypeError("points and origins differ in dtype")
        self.device = points_soa.device
        self.points, self.origins = points_soa, origins_soa
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        handle = ctypes.c_void_p()
        _check(lib().skycell_quadrant_create(ctypes.c_void_p(points_soa.data_ptr()), self.dtype, self.n, self.d,
                                             int(value_bits), ctypes.c_void_p(origins_soa.data_ptr()), self.nq,
                                             ctypes.byref(handle), st))
        self.handle = handle
        self.out_off = np.zeros(self.nq + 1, dtype=np.int64)
        _check(lib().skycell_quadrant_offsets(self.handle, self.out_off.ctypes.data))
        self.out_idx = torch.empty(max(int(self.out_off[-1]), 1), dtype=torch.int32, device=self.device)
        self.out_count = torch.empty(self.nq, dtype=torch.int32, device=self.device)

    def run(self):
        import torch
        st = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _check(lib().skycell_quadrant_run(self.handle, ctypes.c_void_p(self.points.data_ptr()),
                                          ctypes.c_void_p(self.origins.data_ptr()),
                                          ctypes.c_void_p(self.out_idx.data_ptr()),
                                          ctypes.c_void_p(self.out_count.data_ptr()), st))
        return self.out_idx, self.out_count

    def answers(self):
        """Per-query ascending indices (numpy), after run()."""
        idx = self.out_idx.cpu().numpy()
        cnt = self.out_count.cpu().numpy()
        if (cnt < 0).any():
            raise SkycellError(int(cnt[cnt < 0][0]), "a quadrant holds a NaN")
        return [idx[self.out_off[q]:self.out_off[q] + cnt[q]] for q in range(self.nq)]

    def close(self):
        if self.handle:
            _check(lib().skycell_quadrant_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedPlan:
    """Many independent skylines in one graph launch (captured at the first run).

    ns, ds: per-instance point counts and dimensionalities.  The points of all
    instances live in one device buffer of concatenated SoA blocks (see
    ``pack``); results come back per instance as local ascending indices.
    """

    def __init__(self, ns, ds, dtype="f32", value_bits=10, grid_res=None, device="cuda"):
        import numpy as np
        import torch
        self.num = len(ns)
        if len(ds) != self.num:
            raise ValueError("ns and ds differ in length")
        self.ns = np.ascontiguousarray(np.asarray(ns, dtype=np.int64))
        self.ds = np.ascontiguousarray(np.asarray(ds, dtype=np.int32))
        self.dtype = DTYPE_F32 if dtype in ("f32", DTYPE_F32) else DTYPE_U16
        self.device = torch.device(device)
        g = None if grid_res is None else np.ascontiguousarray(np.asarray(grid_res, dtype=np.int32))
        handle = ctypes.c_void_p()
        _check(lib().skycell_batched_plan_create(
            self.num, self.ns.ctypes.data, self.ds.ctypes.data, self.dtype, int(value_bits),
            g.ctypes.data if g is not None else None, ctypes.byref(handle)))
        self.handle = handle
        self.points_off = np.zeros(self.num + 1, dtype=np.int64)
        self.out_off = np.zeros(self.num + 1, dtype=np.int64)
        self.grid_res = np.zeros(self.num, dtype=np.int32)
        _check(lib().skycell_batched_offsets(self.handle, self.points_off.ctypes.data,
                                             self.out_off.ctypes.data, self.grid_res.ctypes.data))
        self.out_idx = torch.empty(max(int(self.out_off[-1]), 1), dtype=torch.int32, device=self.device)
        self.out_count = torch.empty(self.num, dtype=torch.int32, device=self.device)

    def pack(self, arrays):
        """Host arrays [n_b, d_b] -> one device buffer of SoA blocks."""
        import numpy as np
        import torch
        tdt = np.float32 if self.dtype == DTYPE_F32 else np.uint16
        buf = np.empty(max(int(self.points_off[-1]), 1), dtype=tdt)
        for b, a in enumerate(arrays):
            a = np.asarray(a)
            if a.shape != (int(self.ns[b]), int(self.ds[b])) or a.dtype != tdt:
                raise ValueError("instance %d: expected %s array of shape (%d, %d)" %
                                 (b, tdt.__name__, self.ns[b], self.ds[b]))
            buf[self.points_off[b]:self.points_off[b + 1]] = a.T.reshape(-1)
        return torch.from_numpy(buf).to(self.device)

    def run(self, points, stream=None):
        """Enqueue one batched launch over `points` (a packed device buffer)."""
        import torch
        st = stream if stream is not None else torch.cuda.current_stream(self.device).cuda_stream
        _check(lib().skycell_batched_run(self.handle, ctypes.c_void_p(points.data_ptr()),
                                         ctypes.c_void_p(self.out_idx.data_ptr()),
                                         ctypes.c_void_p(self.out_count.data_ptr()), ctypes.c_void_p(st)))

    def results(self):
        """Per-instance skyline indices (numpy int32), after synchronising."""
        counts = self.out_count.cpu().numpy()
        idx = self.out_idx.cpu().numpy()
        out = []
        for b in range(self.num):
            c = int(counts[b])
            if c < 0:
                raise SkycellError(c, "instance %d: device reported %s" % (b, "NaN" if c == E_NAN else "error"))
            out.append(idx[self.out_off[b]:self.out_off[b] + c].copy())
        return out

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().skycell_plan_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------- learned proposer
def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream(device, stream=None):
    import torch
    return ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(device).cuda_stream)


def mlp_num_params(d):
    c = ctypes.c_int64(0)
    _check(lib().skycell_mlp_num_params(int(d), ctypes.byref(c)))
    return c.value


class MLP:
    """Pivot-scoring network 2d -> 64 -> 64 -> 1 on the current device (see
    include/skycell.h for the features, the parameter order and the training
    rule).  Points are [d, n] float32 tensors (SoA); a [d, N] tensor sliced as
    x[:, a:b] is a mini-batch (its leading dimension is taken from the stride).
    """

    def __init__(self, d, grid_res, seed=0, _handle=None):
        self.d, self.grid_res = int(d), int(grid_res)
        if _handle is None:
            h = ctypes.c_void_p()
            _check(lib().skycell_mlp_create(self.d, self.grid_res, ctypes.c_uint64(seed), ctypes.byref(h)))
            _handle = h
        self.handle = _handle
        self.count = mlp_num_params(self.d)

    @staticmethod
    def load(path):
        h = ctypes.c_void_p()
        _check(lib().skycell_mlp_load(path.encode(), ctypes.byref(h)))
        with open(path, "rb") as f:
            f.read(8)
            import struct
            d, g = struct.unpack("<ii", f.read(8))
        return MLP(d, g, _handle=h)

    def save(self, path):
        _check(lib().skycell_mlp_save(self.handle, path.encode()))

    def _host(self, fn, values=None):
        import numpy as np
        buf = np.zeros(self.count, np.float32) if values is None else np.ascontiguousarray(values, np.float32)
        if buf.shape != (self.count,):
            raise ValueError("expected %d parameters" % self.count)
        _check(fn(self.handle, buf.ctypes.data, self.count))
        return buf

    def get_params(self):
        return self._host(lib().skycell_mlp_get_params)

    def set_params(self, values):
        self._host(lib().skycell_mlp_set_params, values)

    def get_grads(self):
        return self._host(lib().skycell_mlp_get_grads)

    def set_grads(self, values):
        self._host(lib().skycell_mlp_set_grads, values)

    @staticmethod
    def _soa(points):
        if points.dim() != 2 or (points.shape[1] > 1 and points.stride(1) != 1):
            raise ValueError("points must be a [d, n] tensor with unit stride along n")
        n = points.shape[1]
        # a single row's stride is arbitrary; any ld >= n addresses it
        return n, points.stride(0) if points.shape[0] > 1 else max(n, 1)

    def score(self, points, out=None, stream=None):
        import torch
        n, ld = self._soa(points)
        out = torch.empty(n, dtype=torch.float32, device=points.device) if out is None else out
        _check(lib().skycell_mlp_score(self.handle, _ptr(points), ld, n, _ptr(out), _stream(points.device, stream)))
        return out

    def backward(self, points, labels, loss_out=None, stream=None):
        n, ld = self._soa(points)
        _check(lib().skycell_mlp_backward(self.handle, _ptr(points), ld, _ptr(labels), n, _ptr(loss_out),
                                          _stream(points.device, stream)))

    def adam_step(self, lr, device="cuda", stream=None):
        import torch
        _check(lib().skycell_mlp_adam_step(self.handle, ctypes.c_float(lr), _stream(torch.device(device), stream)))

    def train_step(self, points, labels, lr, loss_out=None, stream=None):
        n, ld = self._soa(points)
        _check(lib().skycell_mlp_train_step(self.handle, _ptr(points), ld, _ptr(labels), n, ctypes.c_float(lr),
                                            _ptr(loss_out), _stream(points.device, stream)))

    def close(self):
        if getattr(self, "handle", None):
            _check(lib().skycell_mlp_destroy(self.handle))
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def skyline_labels(out_idx, out_count, n, stream=None):
    """uint8 [n] device labels: 1 at the indices of a skyline result."""
    import torch
    labels = torch.empty(max(int(n), 1), dtype=torch.uint8, device=out_idx.device)
    _check(lib().skycell_skyline_labels(_ptr(out_idx), _ptr(out_count), int(n), _ptr(labels),
                                        _stream(out_idx.device, stream)))
    return labels[:int(n)]


def topk(scores, k, stream=None):
    """Indices of the min(k, n) largest scores, largest first, ties by index."""
    import torch
    n = scores.numel()
    kk = min(int(k), n)
    out = torch.empty(max(kk, 1), dtype=torch.int32, device=scores.device)
    _check(lib().skycell_topk(_ptr(scores.contiguous()), n, int(k), _ptr(out), _stream(scores.device, stream)))
    return out[:kk]


def _pivoted(points_soa, grid_res, pivots, mlp, k, return_stats, stream):
    import torch
    if points_soa.dtype != torch.float32 or not points_soa.is_contiguous() or points_soa.dim() != 2:
        raise ValueError("points must be a contiguous float32 [d, n] tensor")
    d, n = points_soa.shape
    dev = points_soa.device
    out_idx = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    out_count = torch.empty(1, dtype=torch.int32, device=dev)
    stats = torch.zeros(NUM_STATS, dtype=torch.int64, device=dev) if return_stats else None
    st = _stream(dev, stream)
    if mlp is None:
        piv = pivots.to(torch.int32).contiguous()
        _check(lib().skycell_compute_with_pivots(_ptr(points_soa), n, d, int(grid_res), _ptr(piv), piv.numel(),
                                                 _ptr(out_idx), _ptr(out_count), _ptr(stats), st))
    else:
        _check(lib().skycell_compute_pivoted(_ptr(points_soa), n, d, int(grid_res), mlp.handle, int(k),
                                             _ptr(out_idx), _ptr(out_count), _ptr(stats), st))
    c = int(out_count.item())
    if c < 0:
        raise SkycellError(c, "device reported %s" % ("NaN in input" if c == E_NAN else "a pivot index out of range"))
    res = out_idx[:c].clone()
    if return_stats:
        return res, dict(zip(STAT_NAMES, (int(v) for v in stats.cpu().tolist())))
    return res


def compute_with_pivots(points_soa, pivots, grid_res=0, return_stats=False, stream=None):
    """Exact skyline of [d, n] float32 points with the given pivot indices as
    a pre-filter (the result equals compute's)."""
    return _pivoted(points_soa, grid_res, pivots, None, 0, return_stats, stream)


def compute_pivoted(points_soa, mlp, k=MAX_PIVOTS, grid_res=0, return_stats=False, stream=None):
    """Exact skyline of [d, n] float32 points with the network's k best points
    as pivots (the result equals compute's)."""
    return _pivoted(points_soa, grid_res, None, mlp, k, return_stats, stream)
