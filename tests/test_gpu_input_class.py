"""The input class (skycell_input_class) the library computes from a strided
sample of its input: the mean correlation of two attributes, from the
per-dimension variances and the variance of the coordinate sum.  Each seeded
generator's data must fall into its own class, at any d, for binary32 and
uint16 inputs; constant and single-attribute inputs are independent."""
import numpy as np
import pytest

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _soa(x):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.from_numpy(np.ascontiguousarray(x.T)).to(torch.device("cuda:0"))


@pytest.mark.parametrize("d", [2, 3, 4, 8, 12, 16])
def test_each_generator_falls_into_its_class(d):
    for cls, dist in enumerate(datagen.DISTRIBUTIONS):
        assert sky.CLASS_NAMES[cls] == dist
        for n in (1_000, 300_000):   # all points, and a strided sample of 65,536
            x = datagen.generate(dist, n, d, seed=40 + d)
            assert sky.input_class(_soa(x)) == cls, (dist, n, d)


def test_uint16_and_degenerate_inputs():
    u = datagen.quantise_u16(datagen.anticorrelated(200_000, 6, seed=3))
    assert sky.input_class(_soa(u)) == sky.CLASS_ANTICORRELATED
    u = datagen.quantise_u16(datagen.correlated(200_000, 6, seed=4))
    assert sky.input_class(_soa(u)) == sky.CLASS_CORRELATED
    assert sky.input_class(_soa(np.full((5_000, 4), 0.5, dtype=np.float32))) == sky.CLASS_INDEPENDENT
    assert sky.input_class(_soa(datagen.anticorrelated(5_000, 1, seed=5))) == sky.CLASS_INDEPENDENT
