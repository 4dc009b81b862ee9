"""The paper's parallel ShrinkKeyCells (Algorithm 3, layer by layer as in
Algorithm 1) on the GPU: every layer's key and candidate cells equal the
oracle's run of the same algorithm (oracle/cells.py) bit for bit, and the
skyline computed with the tree-form prune equals the oracle's skyline (the
tree keeps a superset of Definition 3's survivors; the refine stays exact)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import cells as C
import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def soa(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(DEV)


def morton(c, d, L):
    x = 0
    for k in range(d):
        for b in range(L):
            x |= ((c[k] >> b) & 1) << (b * d + k)
    return x


def bitmap(cells, d, L):
    words = ((1 << (L * d)) + 63) // 64
    out = np.zeros(words, dtype=np.uint64)
    for c in cells:
        x = morton(c, d, L)
        out[x >> 6] |= np.uint64(1) << np.uint64(x & 63)
    return out


@pytest.mark.parametrize("dist,n,d,rho", [
    ("independent", 3000, 2, 5), ("anticorrelated", 4000, 3, 4), ("correlated", 5000, 3, 3),
    ("independent", 2000, 4, 3), ("anticorrelated", 6000, 5, 2), ("independent", 1500, 1, 6),
    ("anticorrelated", 20000, 8, 2), ("anticorrelated", 60000, 6, 2),
])
def test_tree_layers_match_the_oracle_run(dist, n, d, rho):
    x = datagen.generate(dist, n, d, 30 + d if n != 60000 else 50 + d)
    got = sky.shrink_tree_layers(soa(x), rho)

    def layer_cells(i):
        return {tuple(c) for c in oracle.cell_coords(x, 1 << i).tolist()}

    want = C.layers_parallel(layer_cells, rho, d)
    for L in range(1, rho + 1):
        keys = [c for c, t in want[L].items() if t == "key"]
        cand = list(want[L].keys())
        gk, gc = got[L - 1]
        wk, wc = bitmap(keys, d, L), bitmap(cand, d, L)
        if not (np.array_equal(gk, wk) and np.array_equal(gc, wc)):
            diff = []
            for name, a, b in (("key", gk, wk), ("cand", gc, wc)):
                x_ = np.nonzero(np.unpackbits((a ^ b).view(np.uint8), bitorder="little"))[0]
                diff.append((name, x_[:10].tolist(), [int(v) for v in x_[:10] if (a.view(np.uint8)[v >> 3] >> (v & 7)) & 1]))
            raise AssertionError("layer %d differs: %s" % (L, diff))


@pytest.mark.parametrize("dist,n,d,g", [
    ("independent", 50_000, 4, 16), ("anticorrelated", 60_000, 6, 4), ("correlated", 40_000, 3, 32),
    ("anticorrelated", 200_000, 8, 8), ("independent", 100_000, 8, 4),
])
def test_tree_prune_keeps_the_skyline_exact(dist, n, d, g):
    x = datagen.generate(dist, n, d, 50 + d)
    xs = soa(x)
    want = oracle.skyline_sfs(x)
    plain, st0 = sky.compute(xs, grid_res=g, layout="dn", return_stats=True)
    sky.set_cell_prune("tree")
    try:
        got, st1 = sky.compute(xs, grid_res=g, layout="dn", return_stats=True)
    finally:
        sky.set_cell_prune("prefix_or")
    assert np.array_equal(got.cpu().numpy(), want)
    assert np.array_equal(plain.cpu().numpy(), want)
    # the tree's verdicts are one-sided: at least Definition 3's survivors
    assert st1["surviving_cells"] >= st0["surviving_cells"]
    assert st1["survivor_points"] >= st0["survivor_points"]
    # and exactly the non-empty candidate cells of the oracle's run of Algorithm 3
    rho = g.bit_length() - 1
    if d * rho <= 12:
        def layer_cells(i):
            return {tuple(c) for c in oracle.cell_coords(x, 1 << i).tolist()}
        res = C.layers_parallel(layer_cells, rho, d)
        ne = layer_cells(rho)
        assert st1["surviving_cells"] == sum(1 for c in res[rho] if c in ne)


def test_tree_prune_ignored_for_other_grids():
    x = datagen.generate("independent", 20_000, 3, 1)
    sky.set_cell_prune("tree")
    try:
        got = sky.compute(soa(x), grid_res=6, layout="dn")
    finally:
        sky.set_cell_prune("prefix_or")
    assert np.array_equal(got.cpu().numpy(), oracle.skyline_sfs(x))
