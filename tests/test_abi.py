"""The C ABI loads, exports every declared symbol, and rejects bad arguments
before touching the GPU (these tests run on a machine without one)."""
import ctypes
import os
import re

import pytest

import paper_2107_09993_amd as sky

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skycell.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(skycell_\w+)\s*\(", src)))


def test_header_declares_expected_entry_points():
    names = _declared()
    for want in ("skycell_compute", "skycell_compute_u16", "skycell_compute_ws",
                 "skycell_workspace_bytes", "skycell_choose_grid", "skycell_last_error",
                 "skycell_mlp_create", "skycell_mlp_train_step", "skycell_mlp_score",
                 "skycell_topk", "skycell_compute_pivoted", "skycell_compute_with_pivots"):
        assert want in names


def test_library_exports_every_declared_symbol():
    lib = sky.lib()
    for name in _declared():
        assert hasattr(lib, name), name


def test_constants_match_header():
    src = open(HEADER).read()
    assert "SKYCELL_MAX_D 16" in src and sky.MAX_D == 16
    assert "SKYCELL_NUM_STATS 9" in src and sky.NUM_STATS == 9 == len(sky.STAT_NAMES)
    assert "SKYCELL_MAX_PIVOTS 4096" in src and sky.MAX_PIVOTS == 4096
    for name, val in (("SKYCELL_E_INVAL", -1), ("SKYCELL_E_RANGE", -2), ("SKYCELL_E_NOMEM", -3),
                      ("SKYCELL_E_HIP", -4), ("SKYCELL_E_NODEV", -5), ("SKYCELL_E_NAN", -6)):
        assert re.search(r"%s\s*=\s*%d" % (name, val), src)


FAKE = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first


@pytest.mark.parametrize("n,d,g,pts,out_idx,out_count,code", [
    (10, 4, 8, None, FAKE, FAKE, sky.E_INVAL),       # null points
    (10, 4, 8, FAKE, None, FAKE, sky.E_INVAL),       # null out_idx
    (10, 4, 8, FAKE, FAKE, None, sky.E_INVAL),       # null out_count
    (-1, 4, 8, FAKE, FAKE, FAKE, sky.E_INVAL),       # negative n
    (1 << 31, 4, 8, FAKE, FAKE, FAKE, sky.E_INVAL),  # n too large for int32 indices
    (10, 0, 8, FAKE, FAKE, FAKE, sky.E_INVAL),       # d too small
    (10, 17, 8, FAKE, FAKE, FAKE, sky.E_INVAL),      # d too large
    (10, 4, -3, FAKE, FAKE, FAKE, sky.E_INVAL),      # negative grid
    (10, 8, 10, FAKE, FAKE, FAKE, sky.E_RANGE),      # 10^8 cells over budget
    (10, 16, 4, FAKE, FAKE, FAKE, sky.E_RANGE),      # 4^16 cells over budget
])
def test_compute_argument_errors(n, d, g, pts, out_idx, out_count, code):
    lib = sky.lib()
    rc = lib.skycell_compute(pts, n, d, g, out_idx, out_count, None)
    assert rc == code
    assert sky.last_error() != ""


def test_u16_value_bits_checked():
    lib = sky.lib()
    assert lib.skycell_compute_u16(FAKE, 10, 3, 4, 0, FAKE, FAKE, None) == sky.E_RANGE
    assert lib.skycell_compute_u16(FAKE, 10, 3, 4, 17, FAKE, FAKE, None) == sky.E_RANGE


def test_ws_variant_checks_workspace_size_first():
    lib = sky.lib()
    need = sky.workspace_bytes(1000, 4, 8)
    assert need > 0
    rc = lib.skycell_compute_ws(FAKE, sky.DTYPE_F32, 1000, 4, 8, 0, FAKE, FAKE, FAKE, need - 1,
                                None, None)
    assert rc == sky.E_NOMEM
    rc = lib.skycell_compute_ws(FAKE, 7, 1000, 4, 8, 0, FAKE, FAKE, FAKE, need, None, None)
    assert rc == sky.E_INVAL
    rc = lib.skycell_compute_ws(FAKE, sky.DTYPE_F32, 1000, 4, 8, 0, FAKE, FAKE, None, need, None, None)
    assert rc == sky.E_NOMEM
    # misaligned workspace
    rc = lib.skycell_compute_ws(FAKE, sky.DTYPE_F32, 1000, 4, 8, 0, FAKE, FAKE,
                                ctypes.c_void_p(0x1008), need, None, None)
    assert rc == sky.E_INVAL


def test_workspace_bytes_grows_with_n_and_grid():
    a = sky.workspace_bytes(1000, 4, 8)
    b = sky.workspace_bytes(100000, 4, 8)
    c = sky.workspace_bytes(1000, 4, 16)
    assert a < b and a < c
    # layout offsets are increasing, aligned and end at the total
    offs = (ctypes.c_size_t * 13)()
    assert sky.lib().skycell_workspace_layout(1000, 4, 8, 0, offs, 13) == 0
    assert sky.lib().skycell_workspace_layout(1000, 4, 8, 0, offs, 12) == sky.E_INVAL
    vals = list(offs)
    assert vals == sorted(vals) and all(v % 256 == 0 for v in vals)
    assert vals[-1] == a
    with pytest.raises(sky.SkycellError):
        sky.workspace_bytes(10, 20, 2)


def test_choose_grid_respects_budget():
    for d in range(1, 17):
        for n in (1, 100, 10_000, 1_000_000, 10_000_000, 20_000_000):
            g = sky.choose_grid(n, d)
            assert g >= 1
            assert g ** d <= sky.MAX_CELLS
    # the headline shapes
    assert sky.choose_grid(10_000_000, 8) == 8
    assert sky.choose_grid(10_000_000, 6, sky.DTYPE_U16) == 16


def test_tuning_table_roundtrip(tmp_path):
    shipped = os.path.join(os.path.dirname(sky.__file__), "tuning", "mi355x.txt")
    p = tmp_path / "tune.txt"
    # d log2n dtype g [form [parts]]: a five- and a six-column line, and a bad parts value
    p.write_text("# d log2n dtype g form parts\n6 20 0 3\n7 20 0 2 1 8\n5 20 0 2 1 999\n")
    try:
        sky.load_tuning(str(p))
        assert sky.choose_grid(1 << 20, 6) == 3
        assert sky.choose_grid(1 << 20, 7) == 2
        assert sky.choose_grid(1 << 20, 5) == 2
        sky.load_tuning(None)
        # without a table: about two cells per point, 2^18 cells for d = 6
        assert sky.choose_grid(1 << 20, 6) == 8
    finally:
        sky.load_tuning(shipped if os.path.exists(shipped) else None)


def test_class_rows_of_the_tuning_table(tmp_path):
    """Rows tuned on one input class win for that class; other classes fall
    back to the rows chosen over all classes."""
    shipped = os.path.join(os.path.dirname(sky.__file__), "tuning", "mi355x.txt")
    p = tmp_path / "classes.txt"
    p.write_text("# d log2n dtype g form parts class\n8 20 0 3 1 16\n8 20 0 8 1 12 1\n8 20 0 6 0 1 2\n"
                 "8 20 0 5 1 4 7\n")
    try:
        sky.load_tuning(str(p))
        assert sky.choose_config(1_000_000, 8) == (3, "wave", 16)
        assert sky.choose_config(1_000_000, 8, cls=sky.CLASS_INDEPENDENT) == (3, "wave", 16)
        assert sky.choose_config(1_000_000, 8, cls=sky.CLASS_CORRELATED) == (8, "wave", 12)
        assert sky.choose_config(1_000_000, 8, cls=sky.CLASS_ANTICORRELATED) == (6, "lane", 0)
        # a class outside 0..2 in the table is read as "any class": the 7-class
        # line then competes with the first any-class line at the same distance
        assert sky.choose_grid(1_000_000, 8) in (3, 5)
        # rows more than a factor ~2 away in n do not apply to the grid choice
        assert sky.choose_config(1 << 24, 8, cls=sky.CLASS_CORRELATED)[0] == sky.choose_grid(1 << 24, 8)
        lib = sky.lib()
        g, f, q = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        assert lib.skycell_choose_config(10, 8, 0, 3, ctypes.byref(g), ctypes.byref(f), ctypes.byref(q)) == sky.E_INVAL
        assert lib.skycell_choose_config(10, 8, 0, -1, None, ctypes.byref(f), ctypes.byref(q)) == sky.E_INVAL
        c = ctypes.c_int32()
        assert lib.skycell_input_class(None, 0, 10, 8, ctypes.byref(c), None) == sky.E_INVAL
        assert lib.skycell_input_class(FAKE, 0, 0, 8, ctypes.byref(c), None) == sky.E_INVAL
        assert lib.skycell_input_class(FAKE, 0, 10, 17, ctypes.byref(c), None) == sky.E_INVAL
        assert lib.skycell_input_class(FAKE, 5, 10, 8, ctypes.byref(c), None) == sky.E_INVAL
    finally:
        sky.load_tuning(shipped if os.path.exists(shipped) else None)


def test_wave_parts_argument_errors():
    for bad in (-1, 65):
        with pytest.raises(sky.SkycellError) as e:
            sky.set_wave_parts(bad)
        assert e.value.code == sky.E_INVAL
    sky.set_wave_parts(3)
    sky.set_wave_parts(0)


def test_refine_form_argument_errors():
    lib = sky.lib()
    for bad in (-2, 4):
        assert lib.skycell_set_refine_form(bad) == sky.E_INVAL
    for form in sky.REFINE_FORMS:
        sky.set_refine_form(form)
    sky.set_refine_form("auto")


def test_slab_split_argument_errors():
    lib = sky.lib()
    for bad in (-2, 3):
        assert lib.skycell_set_slab_split(bad) == sky.E_INVAL
    for mode in sky.SLAB_SPLIT_MODES:
        sky.set_slab_split(mode)
    sky.set_slab_split("auto")


def test_batched_plan_argument_errors():
    import numpy as np
    lib = sky.lib()
    h = ctypes.c_void_p()
    n = np.asarray([10, 20], dtype=np.int64)
    d = np.asarray([3, 4], dtype=np.int32)
    assert lib.skycell_batched_plan_create(0, n.ctypes.data, d.ctypes.data, 0, 16, None, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_batched_plan_create(2, None, d.ctypes.data, 0, 16, None, ctypes.byref(h)) == sky.E_INVAL
    bad_d = np.asarray([3, 17], dtype=np.int32)
    assert lib.skycell_batched_plan_create(2, n.ctypes.data, bad_d.ctypes.data, 0, 16, None, ctypes.byref(h)) == sky.E_INVAL
    bad_n = np.asarray([10, -1], dtype=np.int64)
    assert lib.skycell_batched_plan_create(2, bad_n.ctypes.data, d.ctypes.data, 0, 16, None, ctypes.byref(h)) == sky.E_INVAL
    g = np.asarray([8, 64], dtype=np.int32)  # 64^4 = 2^24 cells > 2^16 for 20 points
    assert lib.skycell_batched_plan_create(2, n.ctypes.data, d.ctypes.data, 0, 16, g.ctypes.data, ctypes.byref(h)) == sky.E_RANGE
    assert "64 columns in 4 dimensions" in sky.last_error()
    assert lib.skycell_batched_plan_create(2, n.ctypes.data, d.ctypes.data, 1, 0, None, ctypes.byref(h)) == sky.E_RANGE
    assert lib.skycell_batched_plan_create(2, n.ctypes.data, d.ctypes.data, 5, 16, None, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_batched_run(None, FAKE, FAKE, FAKE, None) == sky.E_INVAL
    assert lib.skycell_plan_destroy(None) == sky.E_INVAL


# ---------------------------------------------------------------- learned path
def test_mlp_num_params():
    from oracle import learned
    for d in (1, 3, 10, 16):
        assert sky.mlp_num_params(d) == learned.num_params(d) == 128 * d + 4289
    assert sky.mlp_num_params(10) == 5569
    with pytest.raises(sky.SkycellError):
        sky.mlp_num_params(0)


def test_mlp_create_argument_errors():
    lib = sky.lib()
    h = ctypes.c_void_p()
    assert lib.skycell_mlp_create(0, 4, 1, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_mlp_create(17, 4, 1, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_mlp_create(4, 0, 1, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_mlp_create(4, 4, 1, None) == sky.E_INVAL
    assert lib.skycell_mlp_destroy(None) == sky.OK


def test_mlp_load_rejects_bad_files(tmp_path):
    lib = sky.lib()
    h = ctypes.c_void_p()
    assert lib.skycell_mlp_load(str(tmp_path / "missing.bin").encode(), ctypes.byref(h)) == sky.E_INVAL
    bad = tmp_path / "bad.bin"
    bad.write_bytes(b"NOTANMLP" + bytes(64))
    assert lib.skycell_mlp_load(str(bad).encode(), ctypes.byref(h)) == sky.E_INVAL
    import struct
    short = tmp_path / "short.bin"
    short.write_bytes(b"SKYMLP01" + struct.pack("<iiii", 4, 8, 0, 128 * 4 + 4289) + bytes(16))
    assert lib.skycell_mlp_load(str(short).encode(), ctypes.byref(h)) == sky.E_INVAL
    assert "truncated" in sky.last_error()
    wrong = tmp_path / "wrong.bin"
    wrong.write_bytes(b"SKYMLP01" + struct.pack("<iiii", 4, 8, 0, 99))
    assert lib.skycell_mlp_load(str(wrong).encode(), ctypes.byref(h)) == sky.E_INVAL


def test_pivoted_argument_errors():
    lib = sky.lib()
    # k outside [0, 4096], null pivots, null network: all rejected before any HIP call
    assert lib.skycell_compute_with_pivots(FAKE, 10, 4, 8, FAKE, 4097, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_with_pivots(FAKE, 10, 4, 8, FAKE, -1, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_with_pivots(FAKE, 10, 4, 8, None, 5, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_with_pivots(FAKE, 10, 0, 8, FAKE, 5, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_with_pivots(FAKE, 10, 8, 10, FAKE, 5, FAKE, FAKE, None, None) == sky.E_RANGE
    assert lib.skycell_compute_pivoted(FAKE, 10, 4, 8, None, 16, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_topk(FAKE, 10, 0, FAKE, None) == sky.E_INVAL
    assert lib.skycell_topk(FAKE, 10, 4097, FAKE, None) == sky.E_INVAL
    assert lib.skycell_topk(FAKE, -1, 5, FAKE, None) == sky.E_INVAL
    assert lib.skycell_topk(None, 10, 5, FAKE, None) == sky.E_INVAL
    assert lib.skycell_skyline_labels(FAKE, FAKE, -1, FAKE, None) == sky.E_INVAL
    assert lib.skycell_skyline_labels(None, FAKE, 5, FAKE, None) == sky.E_INVAL
    assert lib.skycell_mlp_score(None, FAKE, 10, 10, FAKE, None) == sky.E_INVAL
    assert lib.skycell_mlp_train_step(None, FAKE, 10, FAKE, 10, ctypes.c_float(0.1), None, None) == sky.E_INVAL


def test_static_entry_point_rejects_sizes_over_its_scratch():
    """skycell_compute_static refuses, on the host, any call whose workspace
    exceeds the fixed scratch array, and validates its arguments first."""
    lib = sky.lib()
    src = open(HEADER).read()
    assert re.search(r"SKYCELL_STATIC_SCRATCH_BYTES \(64u << 20\)", src)
    assert sky.STATIC_SCRATCH_BYTES == 64 << 20
    n = 2_000_000
    assert sky.workspace_bytes(n, 8, 8) > sky.STATIC_SCRATCH_BYTES
    rc = lib.skycell_compute_static(FAKE, sky.DTYPE_F32, n, 8, 8, 0, FAKE, FAKE, None, None)
    assert rc == sky.E_NOMEM
    assert "static scratch" in sky.last_error()
    rc = lib.skycell_compute_static(None, sky.DTYPE_F32, 100, 4, 8, 0, FAKE, FAKE, None, None)
    assert rc == sky.E_INVAL
    rc = lib.skycell_compute_static(FAKE, sky.DTYPE_U16, 100, 4, 8, 17, FAKE, FAKE, None, None)
    assert rc == sky.E_RANGE


def test_dynamic_argument_errors():
    """skycell_dyn_* reject bad arguments before any HIP call."""
    lib = sky.lib()
    h = ctypes.c_void_p()
    assert lib.skycell_dyn_create(0, sky.DTYPE_F32, 100, 10, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(17, sky.DTYPE_F32, 100, 10, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(4, sky.DTYPE_F32, 0, 10, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(4, sky.DTYPE_F32, 1 << 31, 10, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(4, 7, 100, 10, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(4, sky.DTYPE_U16, 100, 0, ctypes.byref(h)) == sky.E_INVAL
    assert lib.skycell_dyn_create(4, sky.DTYPE_F32, 100, 10, None) == sky.E_INVAL
    assert lib.skycell_dyn_insert(None, FAKE, 5, None, None) == sky.E_INVAL
    assert lib.skycell_dyn_delete(None, FAKE, 5, None) == sky.E_INVAL
    assert lib.skycell_dyn_skyline(None, FAKE, FAKE, None) == sky.E_INVAL
    assert lib.skycell_dyn_destroy(None) == sky.OK


def test_quadrant_argument_errors():
    """skycell_quadrant_* reject bad arguments before any HIP call."""
    lib = sky.lib()
    h = ctypes.c_void_p()
    assert lib.skycell_quadrant_create(None, sky.DTYPE_F32, 10, 3, 10, FAKE, 5, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_F32, 10, 3, 10, None, 5, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, 9, 10, 3, 10, FAKE, 5, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_F32, 0, 3, 10, FAKE, 5, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_F32, 10, 17, 10, FAKE, 5, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_F32, 10, 3, 10, FAKE, 0, ctypes.byref(h), None) == sky.E_INVAL
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_U16, 10, 3, 17, FAKE, 5, ctypes.byref(h), None) == sky.E_RANGE
    assert lib.skycell_quadrant_create(FAKE, sky.DTYPE_F32, 10, 3, 10, FAKE, 5, None, None) == sky.E_INVAL
    assert lib.skycell_quadrant_run(None, FAKE, FAKE, FAKE, FAKE, None) == sky.E_INVAL
    assert lib.skycell_quadrant_offsets(None, FAKE) == sky.E_INVAL
    assert lib.skycell_quadrant_destroy(None) == sky.OK


def test_layered_argument_errors():
    lib = sky.lib()
    assert lib.skycell_compute_layered(FAKE, sky.DTYPE_F32, 10, 1, 3, 10, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_layered(FAKE, sky.DTYPE_F32, 10, 9, 3, 10, FAKE, FAKE, None, None) == sky.E_INVAL
    assert lib.skycell_compute_layered(FAKE, sky.DTYPE_F32, 10, 8, 5, 10, FAKE, FAKE, None, None) == sky.E_RANGE
    assert lib.skycell_compute_layered(FAKE, sky.DTYPE_F32, 10, 8, 1, 10, FAKE, FAKE, None, None) == sky.E_RANGE
    assert lib.skycell_compute_layered(None, sky.DTYPE_F32, 10, 8, 4, 10, FAKE, FAKE, None, None) == sky.E_INVAL
