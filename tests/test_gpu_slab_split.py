"""Slab split of the lane refine (the cells with the largest cone-size estimate
get one work item per slab of their lower cone, the cells with one column of
dimension d-1): forced on ("on": the default share of the items; "all": as
many cells as the item array has room for) at sizes the oracle finishes in
seconds, it gives the oracle's skyline, splits cells where the item array has
room (more work items than without it) and falls back to whole cones where it
has none."""
import numpy as np
import pytest
import torch

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

pytestmark = pytest.mark.gpu


def _run(x, g, value_bits=10, pivots=0):
    dev = torch.device("cuda:0")
    n, d = x.shape
    xs = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    if pivots:
        piv = sky.topk(-xs.sum(dim=0), pivots)
        return sky.compute_with_pivots(xs, piv, grid_res=g).cpu().numpy(), None
    s = sky.Skyline(n, d, dtype="f32" if x.dtype == np.float32 else "u16", grid_res=g,
                    value_bits=value_bits, device=dev, stats=True)
    s.run(xs)
    return s.result().cpu().numpy(), s.stats_dict()


def _clustered(n, d, seed):
    """Points in a few dozen tight clusters: cells hold many points each, so
    the item array has room for the split's extra items."""
    rng = np.random.default_rng(seed)
    centres = datagen.anticorrelated(40, d, seed)
    x = centres[rng.integers(0, 40, size=n)] + rng.normal(0, 0.01, size=(n, d)).astype(np.float32)
    return np.clip(x, 0.0, 1.0).astype(np.float32)


# (name, input, grid, whether the split must add items)
CASES = [
    ("clustered_d8_g4", lambda: _clustered(30_000, 8, seed=1), 4, True),
    ("clustered_d4_g16", lambda: _clustered(30_000, 4, seed=2), 16, True),
    # the threshold comes from the occupied cells' cone sizes (survival is not
    # known yet); here the largest cones all belong to dominated clusters
    ("clustered_d2_g64", lambda: _clustered(20_000, 2, seed=3), 64, False),
    ("anti_d7_g4", lambda: datagen.anticorrelated(60_000, 7, seed=4), 4, True),
    ("ind_d5_g8", lambda: datagen.independent(40_000, 5, seed=5), 8, False),
    ("corr_d6_g8", lambda: datagen.correlated(40_000, 6, seed=6), 8, False),
    ("ties_d3_g4", lambda: datagen.small_integers(30_000, 3, seed=7, high=5), 4, False),
    # every point alone in its cell: as many items as slots, no room to split
    ("no_room_d8_g8", lambda: datagen.anticorrelated(3_000, 8, seed=8), 8, False),
    ("tiny_d3", lambda: datagen.independent(7, 3, seed=9), 4, False),
]


@pytest.mark.parametrize("mode", ["on", "all"])
@pytest.mark.parametrize("name,make,g,adds", CASES, ids=[c[0] for c in CASES])
def test_slab_split_matches_oracle(oracle_mod, mode, name, make, g, adds):
    x = make()
    ref = oracle_mod.skyline_sfs(x)
    sky.set_refine_form("lane")
    try:
        sky.set_slab_split("off")
        base, st0 = _run(x, g)
        sky.set_slab_split(mode)
        got, st1 = _run(x, g)
        again, _ = _run(x, g)
    finally:
        sky.set_slab_split("auto")
        sky.set_refine_form("auto")
    assert np.array_equal(base, ref)
    assert np.array_equal(got, ref), (name, mode, len(got), len(ref))
    assert np.array_equal(again, ref)
    assert st1["skyline"] == len(ref)
    assert st1["items"] >= st0["items"]
    if adds and mode == "all":
        assert st1["items"] > st0["items"], (name, st0["items"], st1["items"])
    if name == "no_room_d8_g8":
        assert st1["items"] == st0["items"]


def test_slab_split_u16_and_pivots(oracle_mod):
    """uint16 ties and the pivot pre-filter (which lowers the cells' counts
    after the split is sized) with the split forced on."""
    u = datagen.quantise_u16(_clustered(40_000, 6, seed=10))
    x = datagen.independent(60_000, 8, seed=11)
    sky.set_refine_form("lane")
    sky.set_slab_split("all")
    try:
        got_u, _ = _run(u, 8, value_bits=10)
        got_p, _ = _run(x, 3, pivots=512)
    finally:
        sky.set_slab_split("auto")
        sky.set_refine_form("auto")
    assert np.array_equal(got_u, oracle_mod.skyline_sfs(u))
    assert np.array_equal(got_p, oracle_mod.skyline_sfs(x))
