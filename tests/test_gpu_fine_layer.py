"""Two grid layers beyond the dense cell budget (skycell_compute_layered): the
skyline equals the oracle's, and the fine layer's prune is Definition 3 at
g = 2^rho exactly: the points kept are those of non-dominated non-empty fine
cells (counted against the oracle's cell domination on the same columns), and
the fine survivors respect Equation 14's bound."""
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


def fine_truth(x, g, value_bits=10):
    """Per point: whether its cell at g columns survives Definition 3; the
    numbers of non-empty and surviving cells."""
    cc = oracle.cell_coords(x, g, value_bits=value_bits if x.dtype == np.uint16 else None)
    cells, inv = np.unique(cc, axis=0, return_inverse=True)
    dom = oracle.cells_dominated(cells.astype(np.int32)).astype(bool)
    return ~dom[inv.reshape(-1)], cells.shape[0], int((~dom).sum())


@pytest.mark.parametrize("dist,n,d,rho,u16", [
    ("independent", 40_000, 8, 4, False),     # g = 16: 2^32 fine cells
    ("correlated", 60_000, 8, 4, False),
    ("anticorrelated", 30_000, 8, 4, False),
    ("independent", 50_000, 6, 5, False),     # g = 32: 2^30
    ("anticorrelated", 40_000, 4, 7, False),  # g = 128: 2^28
    ("independent", 30_000, 3, 9, False),     # g = 512: 2^27
    ("anticorrelated", 30_000, 5, 6, True),   # uint16, g = 64: 2^30
    ("independent", 20_000, 2, 14, False),    # g = 16384: 2^28
])
def test_layered_prune_is_definition_3_at_the_fine_grid(dist, n, d, rho, u16):
    x = datagen.generate(dist, n, d, 70 + d)
    if u16:
        x = datagen.quantise_u16(x)
    got, st = sky.compute_layered(soa(x), rho, return_stats=True)
    assert np.array_equal(got.cpu().numpy(), oracle.skyline_sfs(x))
    keep, ne_cells, surv_cells = fine_truth(x, 1 << rho)
    assert st["nonempty_cells"] == ne_cells
    assert st["surviving_cells"] == surv_cells
    assert st["survivor_points"] == int(keep.sum())
    g = 1 << rho
    assert surv_cells <= g ** d - (g - 1) ** d


def test_layered_refuses_what_it_cannot_hold():
    x = soa(datagen.generate("independent", 1000, 8, 1))
    with pytest.raises(sky.SkycellError):
        sky.compute_layered(x, 5)   # 2^40 fine cells
    with pytest.raises(sky.SkycellError):
        sky.compute_layered(soa(datagen.generate("independent", 1000, 9, 1)), 3)   # d > 8
