"""Quadrant skyline queries (Section VII-B3): every query's answer equals the
CPU oracle's skyline of the points in the origin's closed top-right quadrant,
byte for byte as ascending indices."""
import hashlib
import json
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_quadrant_goldens as QG  # noqa: E402


def soa(a):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).T)).to(DEV)


def oracle_answer(x, o):
    ids = np.nonzero((x >= o).all(axis=1))[0]
    if ids.size == 0:
        return ids.astype(np.int32)
    return ids[oracle.skyline_sfs(x[ids])].astype(np.int32)


def run_queries(x, origins, value_bits=10):
    qq = sky.QuadrantQueries(soa(x), soa(origins), value_bits=value_bits)
    qq.run()
    got = qq.answers()
    sizes = np.diff(qq.out_off)
    qq.close()
    return got, sizes


@pytest.mark.parametrize("dist,n,d,nq,u16", [
    ("independent", 5000, 3, 300, False),
    ("anticorrelated", 8000, 4, 200, False),
    ("correlated", 6000, 5, 150, False),
    ("anticorrelated", 7000, 3, 200, True),
])
def test_quadrant_small_against_oracle(dist, n, d, nq, u16):
    x = datagen.generate(dist, n, d, 11 + d)
    rng = np.random.default_rng(n)
    o = rng.random((nq, d), dtype=np.float32) * 0.8
    if u16:
        x = datagen.quantise_u16(x)
        o = datagen.quantise_u16(o)
    # edge origins: a data point itself (closed quadrant), the zero origin (all
    # points), an origin above every point (empty quadrant)
    o[0] = x[17]
    o[1] = 0
    o[2] = 1023 if u16 else 2.0
    if not u16:
        o[3] = -0.0
    got, sizes = run_queries(x, o)
    for q in range(nq):
        want = oracle_answer(x, o[q])
        assert np.array_equal(got[q], want), (q, got[q].size, want.size)
        assert sizes[q] == int((x >= o[q]).all(axis=1).sum())
    assert got[2].size == 0
    assert 17 in set(np.nonzero((x >= o[0]).all(axis=1))[0])


def test_quadrant_10000_queries_against_stored_oracle_answers():
    """The workload of the paper's quadrant experiment: 10,000 random origins
    on one data set (independent, n = 10^5, d = 4); every answer byte-equal to
    the oracle's (tests/golden/quadrants.json, written by
    tests/golden/make_quadrant_goldens.py from the oracle alone)."""
    gold = json.load(open(os.path.join(HERE, "golden", "quadrants.json")))
    x, o = QG.make_data(gold)
    assert QG.sha(x) == gold["data_sha256"] and QG.sha(o) == gold["origins_sha256"]
    got, sizes = run_queries(x, o)
    assert sizes.tolist() == gold["quadrant_sizes"]
    if QG.digest(got) != gold["answers_sha256"]:
        bad = [q for q in range(len(got)) if got[q].size != gold["skyline_sizes"][q]]
        if not bad:
            ref = QG.answers(x, o)
            bad = [q for q in range(len(got)) if not np.array_equal(got[q], ref[q][0])]
        raise AssertionError("queries differing from the oracle: %s" % bad[:20])


def test_quadrant_rerun_and_nan_origin():
    x = datagen.generate("independent", 3000, 2, 5)
    o = np.random.default_rng(2).random((50, 2), dtype=np.float32)
    qq = sky.QuadrantQueries(soa(x), soa(o))
    qq.run()
    first = [a.copy() for a in qq.answers()]
    qq.run()
    second = qq.answers()
    assert all(np.array_equal(a, b) for a, b in zip(first, second))
    qq.close()
    o[7, 1] = np.nan
    with pytest.raises(sky.SkycellError):
        sky.QuadrantQueries(soa(x), soa(o))
