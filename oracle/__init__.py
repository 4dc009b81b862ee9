"""CPU oracle for the SkyCell exact skyline (Definitions 1-2, Section III).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(``paper_2107_09993_amd``) never does, and the two share no code.

* ``skyline_bruteforce`` (O1), ``skyline_sfs`` (O2) and ``skyline_kdtree`` (O3,
  an orthant-emptiness test on a k-d tree, for inputs of 10^6 points and more)
  come from the C file ``skyline_oracle.c`` compiled with gcc by :func:`build`.
* ``skyline_pure_python`` is a third, tiny implementation of the definition for
  exhaustive checks on very small inputs.
* ``cells`` holds the cell-level definitions (Definitions 3-6, Equations 5-14).

Points are row-major ``[n, d]`` numpy arrays (float32 or uint16).  Every function
returns ascending int32 indices of the skyline points, all exact copies included.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "skyline_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "libskyline_oracle.so")
_lib = None

E_NAN = -6


def build(force=False):
    """Compile the C oracle with gcc (no fast-math, no FMA contraction)."""
    if os.path.exists(_LIB_PATH) and not force:
        if os.path.getmtime(_LIB_PATH) >= os.path.getmtime(_SRC):
            return _LIB_PATH
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-pthread", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64, i32, p = ctypes.c_int64, ctypes.c_int, ctypes.c_void_p
    for name in ("orc_skyline_brute_f32", "orc_skyline_sfs_f32", "orc_skyline_kdtree_f32",
                 "orc_skyline_brute_u16", "orc_skyline_sfs_u16", "orc_skyline_kdtree_u16"):
        f = getattr(lib, name)
        f.argtypes = [p, i64, i32, p, i32]
        f.restype = i64
    for name in ("orc_is_skyline_f32", "orc_is_skyline_u16"):
        f = getattr(lib, name)
        f.argtypes = [p, i64, i32, p, i64, p, i32]
        f.restype = i32
    lib.orc_cell_coords_f32.argtypes = [p, i64, i32, i32, p]
    lib.orc_cell_coords_f32.restype = i32
    lib.orc_cell_coords_u16.argtypes = [p, i64, i32, i32, i32, p]
    lib.orc_cell_coords_u16.restype = i32
    lib.orc_cells_dominated.argtypes = [p, i64, i32, p]
    lib.orc_cells_dominated.restype = i32
    lib.orc_dominates_f32.argtypes = [p, p, i32]
    lib.orc_dominates_f32.restype = i32
    _lib = lib
    return lib


def default_threads():
    return max(1, len(os.sched_getaffinity(0)))


def _prep(points):
    a = np.ascontiguousarray(points)
    if a.ndim != 2:
        raise ValueError("points must be [n, d]")
    if a.dtype == np.float32:
        return a, "f32"
    if a.dtype == np.uint16:
        return a, "u16"
    raise TypeError("points must be float32 or uint16")


def _run(kind, points, nthreads):
    a, t = _prep(points)
    n, d = a.shape
    out = np.empty(max(n, 1), dtype=np.int32)
    lib = _load()
    fn = getattr(lib, "orc_skyline_%s_%s" % (kind, t))
    m = fn(a.ctypes.data, n, d, out.ctypes.data, nthreads or default_threads())
    if m == E_NAN:
        raise ValueError("NaN in input")
    if m < 0:
        raise RuntimeError("oracle error %d" % m)
    return out[:m].copy()


def skyline_bruteforce(points, nthreads=None):
    """O1: the definition, O(n^2 d)."""
    return _run("brute", points, nthreads)


def skyline_sfs(points, nthreads=None):
    """O2: sort-first skyline with an exact linear-extension key."""
    return _run("sfs", points, nthreads)


def skyline_kdtree(points, nthreads=None):
    """O3: for each point, is the closed lower orthant {q <= p} free of points
    other than copies of p?  Answered on a k-d tree with bounding boxes."""
    return _run("kdtree", points, nthreads)


def is_skyline(points, indices, nthreads=None):
    """Per-index brute force: for each index i, is points[i] undominated by all points?"""
    a, t = _prep(points)
    n, d = a.shape
    idx = np.ascontiguousarray(np.asarray(indices, dtype=np.int64))
    res = np.zeros(max(idx.size, 1), dtype=np.uint8)
    lib = _load()
    fn = getattr(lib, "orc_is_skyline_%s" % t)
    rc = fn(a.ctypes.data, n, d, idx.ctypes.data, idx.size, res.ctypes.data,
            nthreads or default_threads())
    if rc == E_NAN:
        raise ValueError("NaN in input")
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)
    return res[:idx.size].astype(bool)


def cell_coords(points, g, value_bits=None):
    """Equation 1 with g columns per dimension; returns int32 [n, d] coordinates."""
    a, t = _prep(points)
    n, d = a.shape
    out = np.empty((max(n, 1), d), dtype=np.int32)
    lib = _load()
    if t == "f32":
        rc = lib.orc_cell_coords_f32(a.ctypes.data, n, d, g, out.ctypes.data)
    else:
        rc = lib.orc_cell_coords_u16(a.ctypes.data, n, d, g, value_bits or 16, out.ctypes.data)
    if rc == E_NAN:
        raise ValueError("NaN in input")
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)
    return out[:n]


def cells_dominated(cells):
    """Definition 3 flags for a list of distinct non-empty cells (int32 [m, d])."""
    c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32))
    m, d = c.shape
    out = np.zeros(max(m, 1), dtype=np.uint8)
    rc = _load().orc_cells_dominated(c.ctypes.data, m, d, out.ctypes.data)
    if rc != 0:
        raise RuntimeError("oracle error %d" % rc)
    return out[:m].astype(bool)


def dominates(a, b):
    """Definition 1 for two float32 points."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    y = np.ascontiguousarray(np.asarray(b, dtype=np.float32))
    return bool(_load().orc_dominates_f32(x.ctypes.data, y.ctypes.data, x.size))


def skyline_pure_python(points):
    """Definition 2 in pure Python; only for tiny inputs."""
    pts = [tuple(float(v) for v in row) for row in np.asarray(points)]
    out = []
    for i, p in enumerate(pts):
        dominated = False
        for j, q in enumerate(pts):
            if j != i and all(a <= b for a, b in zip(q, p)) and any(a < b for a, b in zip(q, p)):
                dominated = True
                break
        if not dominated:
            out.append(i)
    return np.asarray(out, dtype=np.int32)
