"""The two-pass scatter (inputs of 2^20 points and more).

Above 2^20 points the library stages the surviving points by ranges of cells
before writing them to their sorted positions.  These tests check the sorted
arrays it leaves in the workspace against their definition (every surviving
point at position start(cell) + rank, with its order-preserving keys, its
packed 7-bit screening columns and its original index), and the skyline
against the CPU oracle, for float32 and uint16 inputs, with the pivot
pre-filter removing points, and for grids with fewer cells than buckets.
"""
import numpy as np
import pytest

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TWO_PASS_MIN = 1 << 20


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _f32_key(x):
    """Order-preserving integer key of binary32 values (-0.0 maps to +0.0's key)."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).copy()
    b[b == 0x80000000] = 0
    neg = (b & 0x80000000) != 0
    return np.where(neg, ~b, b | np.uint32(0x80000000)).astype(np.uint32)


def _fine_cols(x, value_bits):
    """7-bit screening column of every coordinate: floor(x * 128) in binary32,
    clamped to [0, 127]; uint16 values v map to (v * 128) >> value_bits."""
    if x.dtype == np.float32:
        c = np.floor(x * np.float32(128)).astype(np.float64)
        c = np.where(np.isfinite(c), c, 0)
        return np.clip(c, 0, 127).astype(np.uint64)
    return np.minimum((x.astype(np.uint64) * 128) >> np.uint64(value_bits), 127).astype(np.uint64)


def _run(x, g, value_bits=10):
    dev = _dev()
    n, d = x.shape
    dtype = "f32" if x.dtype == np.float32 else "u16"
    s = sky.Skyline(n, d, dtype=dtype, grid_res=g, value_bits=value_bits, device=dev, stats=True)
    s.run(torch.from_numpy(np.ascontiguousarray(x.T)).to(dev))
    out = s.result().cpu().numpy()
    st = s.stats_dict()
    ws = s.workspace.cpu().numpy()
    offs = sky.workspace_layout(n, d, g, dtype=sky.DTYPE_F32 if dtype == "f32" else sky.DTYPE_U16)
    return out, st, ws, offs


def _check_sorted_arrays(x, g, ws, offs, st, value_bits=10):
    n, d = x.shape
    r = int(np.ceil(np.log2(g))) if g > 1 else 0
    cells = 1 << (r * d)
    fw = (d + 7) // 8
    cell_of = ws[offs[0]:offs[0] + 4 * n].view(np.uint32).astype(np.int64)
    rank = ws[offs[1]:offs[1] + 4 * n].view(np.uint32).astype(np.int64)
    rec = ws[offs[4]:offs[4] + 8 * (cells + 1)].view(np.uint64)
    S = int(st["survivor_points"])
    keys = ws[offs[5]:offs[5] + 4 * n * d].view(np.uint32).reshape(n, d)[:S]
    fkeys = ws[offs[6]:offs[6] + 8 * n * fw].view(np.uint64).reshape(n, fw)[:S]
    sidx = ws[offs[7]:offs[7] + 4 * n].view(np.int32)[:S].astype(np.int64)

    surv = (rec[cell_of] >> np.uint64(63)).astype(bool)
    live = np.nonzero(surv)[0]
    assert live.size == S
    # positions: start of the point's cell + its rank, a permutation of [0, S)
    start = (rec[cell_of[live]] & np.uint64(0xFFFFFFFF)).astype(np.int64)
    pos = start + rank[live]
    assert np.array_equal(np.sort(pos), np.arange(S))
    assert np.array_equal(sidx[pos], live)
    # keys and screening columns of every sorted point
    xs = x[live]
    want_keys = _f32_key(xs) if x.dtype == np.float32 else xs.astype(np.uint32)
    assert np.array_equal(keys[pos], want_keys)
    cols = _fine_cols(xs, value_bits)
    want_f = np.zeros((live.size, fw), dtype=np.uint64)
    for k in range(d):
        want_f[:, k // 8] |= cols[:, k] << np.uint64(8 * (k % 8))
    assert np.array_equal(fkeys[pos], want_f)


@pytest.mark.parametrize("n,d,g,dist", [
    (TWO_PASS_MIN, 5, 8, "independent"),        # exactly at the threshold
    (1_300_001, 6, 6, "independent"),           # ragged n, non-power-of-two grid
    (1_100_003, 5, 2, "correlated"),            # 32 cells: fewer cells than buckets
    (TWO_PASS_MIN + 5, 16, 2, "correlated"),    # widest rows (d = 16)
    (TWO_PASS_MIN + 5, 1, 64, "independent"),   # narrowest rows, one skyline point
    (TWO_PASS_MIN + 5, 2, 32, "independent"),
    (TWO_PASS_MIN + 5, 3, 16, "anticorrelated"),
])
def test_sorted_arrays_f32(oracle_mod, n, d, g, dist):
    x = datagen.generate(dist, n, d, seed=11)
    out, st, ws, offs = _run(x, g)
    _check_sorted_arrays(x, g, ws, offs, st)
    assert np.array_equal(out, oracle_mod.skyline_sfs(x))


def test_sorted_arrays_u16_ties(oracle_mod):
    """uint16 coordinates in 0..255 (value_bits 8): duplicates and equal
    coordinates everywhere."""
    x = datagen.quantise_u16(datagen.anticorrelated(1_200_000, 4, seed=12), levels=256)
    out, st, ws, offs = _run(x, 8, value_bits=8)
    _check_sorted_arrays(x, 8, ws, offs, st, value_bits=8)
    assert np.array_equal(out, oracle_mod.skyline_sfs(x))


def test_below_threshold_unchanged(oracle_mod):
    """One point below the threshold the one-pass scatter runs; same checks."""
    x = datagen.independent(TWO_PASS_MIN - 1, 5, seed=13)
    out, st, ws, offs = _run(x, 8)
    _check_sorted_arrays(x, 8, ws, offs, st)
    assert np.array_equal(out, oracle_mod.skyline_sfs(x))


def test_pivot_prefilter_two_pass(oracle_mod):
    """Pivots remove points before the scatter (their rank is the removed mark):
    the skyline still equals the oracle's above the threshold."""
    dev = _dev()
    x = datagen.correlated(1_250_000, 6, seed=14)
    xs = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    piv = sky.topk(-xs.sum(dim=0), 4096)
    got, st = sky.compute_with_pivots(xs, piv, return_stats=True)
    ref = oracle_mod.skyline_sfs(x)
    assert np.array_equal(got.cpu().numpy(), ref)
    assert st["pivot_removed"] > 0
