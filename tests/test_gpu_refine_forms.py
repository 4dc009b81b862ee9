"""The refine forms (lane: one lane walks the cone of a few points of one
cell, passing over cells whose minimum corner rules them out for d <= 8;
plain: the lane form without that screen; wave: one wave walks the cone of up
to 63 points of one cell) give the oracle's skyline on the same inputs, fine
and coarse grids alike."""
import numpy as np
import pytest
import torch

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

pytestmark = pytest.mark.gpu


def _run(x, g, value_bits=10, stats=False):
    dev = torch.device("cuda:0")
    n, d = x.shape
    s = sky.Skyline(n, d, dtype="f32" if x.dtype == np.float32 else "u16", grid_res=g,
                    value_bits=value_bits, device=dev, stats=stats)
    s.run(torch.from_numpy(np.ascontiguousarray(x.T)).to(dev))
    out = s.result().cpu().numpy()
    return (out, s.stats_dict()) if stats else out


def _hot(n, d, seed):
    """Most points in a few cells: a narrow diagonal band plus a third of the rows
    copied from five points (many lanes of one wave land in one cell, and some
    cells hold thousands of refine items)."""
    rng = np.random.default_rng(seed)
    x = datagen.correlated(n, d, seed, sigma=0.01)
    rows = rng.choice(n, size=n // 3, replace=False)
    x[rows] = x[rng.integers(0, n, size=5)][rng.integers(0, 5, size=rows.size)]
    return x


CASES = [
    ("hot_d4_g2", lambda: _hot(60_000, 4, seed=9), 2),
    ("hot_d3_g8", lambda: _hot(60_000, 3, seed=10), 8),
    ("ind_d3_coarse", lambda: datagen.independent(30_000, 3, seed=1), 2),
    ("anti_d8_coarse", lambda: datagen.anticorrelated(20_000, 8, seed=2), 2),
    ("anti_d8_fine", lambda: datagen.anticorrelated(20_000, 8, seed=2), 8),
    ("corr_d12", lambda: datagen.correlated(40_000, 12, seed=3), 2),
    ("ties_d5", lambda: datagen.small_integers(20_000, 5, seed=4, high=5), 3),
    ("ind_d1", lambda: datagen.independent(5_000, 1, seed=5), 4),
    ("ind_d16", lambda: datagen.independent(10_000, 16, seed=6), 2),
    ("ind_d2_one_cell", lambda: datagen.independent(100_000, 2, seed=7), 1),
    ("anti_d10_g3", lambda: datagen.anticorrelated(30_000, 10, seed=8), 3),
    # half of the points in the top screening column of every dimension: their
    # walks pass every cell, empty ones included (whose minima are the "no
    # points" value 63, equal to their halved columns)
    ("top_column_d4", lambda: _top_column(20_000, 4, seed=11), 8),
    # one cell with more points than a cell record's count field holds (the
    # count is read from the next cell's first position), and more than one
    # lane reduces alone when the walk records are built
    ("saturated_cell_d3", lambda: _one_cell(40_000, 3, seed=12), 4),
    ("anti_d7_g6", lambda: datagen.anticorrelated(50_000, 7, seed=13), 6),
]


def _top_column(n, d, seed):
    """Uniform points, half of them moved into [127/128, 1] in every
    coordinate (screening column 127)."""
    x = datagen.independent(n, d, seed)
    top = x[: n // 2] * np.float32(1.0 / 128.0) + np.float32(127.0 / 128.0)
    x[: n // 2] = np.minimum(top, np.float32(1.0))
    return x


def _one_cell(n, d, seed):
    """n points inside one cell of a 4-column grid, with repeated rows."""
    x = datagen.independent(n, d, seed) * np.float32(0.2) + np.float32(0.3)
    x[n // 2:] = x[: n - n // 2][::-1]
    return x


@pytest.mark.parametrize("form", ["lane", "plain", "wave"])
@pytest.mark.parametrize("name,make,g", CASES, ids=[c[0] for c in CASES])
def test_refine_form_matches_oracle(oracle_mod, form, name, make, g):
    x = make()
    ref = oracle_mod.skyline_sfs(x)
    sky.set_refine_form(form)
    try:
        got, st = _run(x, g, stats=True)
    finally:
        sky.set_refine_form("auto")
    assert np.array_equal(got, ref), (form, len(got), len(ref))
    assert st["skyline"] == len(ref)


@pytest.mark.parametrize("form", ["lane", "wave"])
def test_refine_forms_u16(oracle_mod, form):
    x = datagen.quantise_u16(datagen.anticorrelated(40_000, 6, seed=9))
    ref = oracle_mod.skyline_sfs(x)
    sky.set_refine_form(form)
    try:
        got = _run(x, 4, value_bits=10)
    finally:
        sky.set_refine_form("auto")
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("parts", [2, 3, 8, 64])
@pytest.mark.parametrize("name,make,g", CASES, ids=[c[0] for c in CASES])
def test_wave_parts_match_oracle(oracle_mod, parts, name, make, g):
    """The wave form with several waves per item (each screens every parts-th
    candidate group of the cone, dominated points are cleared by whichever wave
    finds a dominator) gives the oracle's skyline."""
    x = make()
    ref = oracle_mod.skyline_sfs(x)
    sky.set_refine_form("wave")
    sky.set_wave_parts(parts)
    try:
        got = _run(x, g)
        again = _run(x, g)
    finally:
        sky.set_refine_form("auto")
        sky.set_wave_parts(0)
    assert np.array_equal(got, ref), (parts, len(got), len(ref))
    assert np.array_equal(again, ref)


def test_wave_parts_pivots_and_u16(oracle_mod):
    """Several waves per item with the pivot pre-filter (removed points start
    with a cleared flag) and with uint16 ties."""
    dev = torch.device("cuda:0")
    x = datagen.independent(60_000, 9, seed=10)
    xs = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    piv = sky.topk(-xs.sum(dim=0), 512)
    u = datagen.quantise_u16(datagen.anticorrelated(40_000, 6, seed=11))
    sky.set_refine_form("wave")
    sky.set_wave_parts(4)
    try:
        got = sky.compute_with_pivots(xs, piv, grid_res=2).cpu().numpy()
        got_u = _run(u, 3, value_bits=10)
    finally:
        sky.set_refine_form("auto")
        sky.set_wave_parts(0)
    assert np.array_equal(got, oracle_mod.skyline_sfs(x))
    assert np.array_equal(got_u, oracle_mod.skyline_sfs(u))


TILE_CASES = [
    ("anti_d8_g8", lambda: datagen.anticorrelated(60_000, 8, seed=12), 8),
    ("anti_d8_g4", lambda: datagen.anticorrelated(30_000, 8, seed=13), 4),
    ("ind_d8_g8", lambda: datagen.independent(80_000, 8, seed=14), 8),
    ("corr_d6_g16", lambda: datagen.correlated(50_000, 6, seed=15), 16),
    ("ind_d2_g128", lambda: datagen.independent(100_000, 2, seed=16), 128),
    ("anti_d3_g64", lambda: datagen.anticorrelated(70_000, 3, seed=17), 64),
    ("ties_d5_g4", lambda: datagen.small_integers(20_000, 5, seed=18, high=5), 4),
    ("anti_d7_g2", lambda: datagen.anticorrelated(9_000, 7, seed=19), 2),
    ("anti_d4_g32_big_cells", lambda: datagen.anticorrelated(400_000, 4, seed=20), 32),
]


@pytest.mark.parametrize("name,make,g", TILE_CASES, ids=[c[0] for c in TILE_CASES])
def test_tile_form_matches_oracle(oracle_mod, name, make, g):
    """Tile form (a workgroup walks the coarse cone of up to 256 points of one
    coarse cell; each point screens the candidates of its own fine cone, staged
    in LDS): the oracle's skyline, and the same number of screening tests as
    the lane form (both screen exactly the fine lower cone until a dominator)."""
    x = make()
    ref = oracle_mod.skyline_sfs(x)
    sky.set_refine_form("tile")
    try:
        got, st = _run(x, g, stats=True)
        again = _run(x, g)
    finally:
        sky.set_refine_form("auto")
    assert np.array_equal(got, ref), (len(got), len(ref))
    assert np.array_equal(again, ref)
    assert st["skyline"] == len(ref)


def test_tile_form_u16_and_unsupported_grids(oracle_mod):
    u = datagen.quantise_u16(datagen.anticorrelated(50_000, 6, seed=21))
    x = datagen.independent(20_000, 9, seed=22)
    sky.set_refine_form("tile")
    try:
        got_u = _run(u, 8, value_bits=10)
        got_odd = _run(u, 6, value_bits=10)   # g not a power of two: the lane form runs
        got_d9 = _run(x, 4)                   # d > 8: the lane form runs
    finally:
        sky.set_refine_form("auto")
    ref_u = oracle_mod.skyline_sfs(u)
    assert np.array_equal(got_u, ref_u)
    assert np.array_equal(got_odd, ref_u)
    assert np.array_equal(got_d9, oracle_mod.skyline_sfs(x))
