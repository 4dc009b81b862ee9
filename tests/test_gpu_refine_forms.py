"""Both refine forms (lane: one lane walks the cone of a few points of one
cell; wave: one wave walks the cone of up to 63 points of one cell) give the
oracle's skyline on the same inputs, fine and coarse grids alike."""
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


CASES = [
    ("ind_d3_coarse", lambda: datagen.independent(30_000, 3, seed=1), 2),
    ("anti_d8_coarse", lambda: datagen.anticorrelated(20_000, 8, seed=2), 2),
    ("anti_d8_fine", lambda: datagen.anticorrelated(20_000, 8, seed=2), 8),
    ("corr_d12", lambda: datagen.correlated(40_000, 12, seed=3), 2),
    ("ties_d5", lambda: datagen.small_integers(20_000, 5, seed=4, high=5), 3),
    ("ind_d1", lambda: datagen.independent(5_000, 1, seed=5), 4),
    ("ind_d16", lambda: datagen.independent(10_000, 16, seed=6), 2),
    ("ind_d2_one_cell", lambda: datagen.independent(100_000, 2, seed=7), 1),
    ("anti_d10_g3", lambda: datagen.anticorrelated(30_000, 10, seed=8), 3),
]


@pytest.mark.parametrize("form", ["lane", "wave"])
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
