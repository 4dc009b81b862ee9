"""Parity of the batched path (a graph of the single-instance path over many instances)
with the CPU oracle, instance by instance."""
import numpy as np
import pytest

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _instances(count, seed, n_lo, n_hi, d_lo=1, d_hi=16):
    rng = np.random.default_rng(seed)
    shapes = []
    for b in range(count):
        n = int(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))
        d = int(rng.integers(d_lo, d_hi + 1))
        dist = datagen.DISTRIBUTIONS[int(rng.integers(0, 3))]
        shapes.append((n, d, dist, 1000 + b))
    return shapes


def test_graph_batched_mixed_small_all_instances(oracle_mod):
    dev = _dev()
    shapes = _instances(60, 0, 1, 6000)
    shapes += [(0, 3, "independent", 7), (1, 5, "anticorrelated", 8), (2, 1, "correlated", 9)]
    arrays = [datagen.generate(dist, n, d, seed) for n, d, dist, seed in shapes]
    plan = sky.BatchedPlan([a.shape[0] for a in arrays], [a.shape[1] for a in arrays], device=dev)
    buf = plan.pack(arrays)
    plan.run(buf)
    got = plan.results()
    refs = [oracle_mod.skyline_sfs(a) for a in arrays]
    for b, (g, r) in enumerate(zip(got, refs)):
        assert np.array_equal(g, r), "instance %d (n=%d, d=%d)" % (b, len(arrays[b]), arrays[b].shape[1])
    # replaying the captured graph gives the same result (control words reset in-kernel)
    for _ in range(2):
        plan.out_idx.fill_(-7)
        plan.run(buf)
        again = plan.results()
        assert all(np.array_equal(a, r) for a, r in zip(again, refs))
    # a different points buffer rebinds the graph
    arrays2 = [datagen.generate("independent", a.shape[0], a.shape[1], 77 + i) for i, a in enumerate(arrays)]
    buf2 = plan.pack(arrays2)
    plan.run(buf2)
    got2 = plan.results()
    for a, g in zip(arrays2, got2):
        assert np.array_equal(g, oracle_mod.skyline_sfs(a))
    plan.close()


def test_graph_batched_explicit_grids_and_u16(oracle_mod):
    dev = _dev()
    rng = np.random.default_rng(3)
    arrays = [rng.integers(0, 16, size=(int(n), int(d))).astype(np.uint16)
              for n, d in zip(rng.integers(1, 4000, size=30), rng.integers(2, 9, size=30))]
    grids = [int(g) for g in rng.integers(1, 5, size=30)]  # within 2^20 cells at d <= 8
    plan = sky.BatchedPlan([a.shape[0] for a in arrays], [a.shape[1] for a in arrays], dtype="u16",
                           value_bits=4, grid_res=grids, device=dev)
    assert list(plan.grid_res) == grids
    plan.run(plan.pack(arrays))
    for a, g in zip(arrays, plan.results()):
        assert np.array_equal(g, oracle_mod.skyline_sfs(a))
    plan.close()


def test_graph_batched_nan_instance(oracle_mod):
    dev = _dev()
    a = datagen.independent(500, 3, seed=1)
    b = datagen.independent(700, 4, seed=2)
    b[5, 1] = np.nan
    plan = sky.BatchedPlan([500, 700], [3, 4], device=dev)
    plan.run(plan.pack([a, b]))
    torch.cuda.synchronize()
    counts = plan.out_count.cpu().numpy()
    assert counts[1] == sky.E_NAN
    assert counts[0] == len(oracle_mod.skyline_sfs(a))
    plan.close()


def test_graph_batched_merge_law(oracle_mod):
    """sky(A1 u ... u A8) = sky(sky(A1) u ... u sky(A8)): the parts' skylines from
    one batched launch, merged and reduced by the single-instance path, give the
    skyline of the whole input (and the oracle's)."""
    dev = _dev()
    x = datagen.anticorrelated(60_000, 5, seed=31)
    cuts = np.sort(np.random.default_rng(31).choice(np.arange(1, len(x)), 7, replace=False))
    parts = np.split(np.arange(len(x)), cuts)
    plan = sky.BatchedPlan([len(p) for p in parts], [5] * len(parts), device=dev)
    plan.run(plan.pack([np.ascontiguousarray(x[p]) for p in parts]))
    kept = np.concatenate([p[r] for p, r in zip(parts, plan.results())])
    plan.close()
    merged = torch.from_numpy(np.ascontiguousarray(x[kept].T)).to(dev)
    again = kept[sky.compute(merged, layout="dn").cpu().numpy()]
    whole = sky.compute(torch.from_numpy(np.ascontiguousarray(x.T)).to(dev), layout="dn").cpu().numpy()
    ref = oracle_mod.skyline_sfs(x)
    assert np.array_equal(np.sort(again), ref)
    assert np.array_equal(whole, ref)
