"""Pins for the CPU oracle: values the paper prints, closed forms, invariants,
special cases with textbook answers and brute force on tiny inputs.

None of these runs on the GPU; they establish that the oracle is right before it
is used to check the HIP path.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

from oracle import cells as C
from paper_2107_09993_amd import datagen

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _all_impls(oracle_mod, pts):
    out = [oracle_mod.skyline_bruteforce(pts), oracle_mod.skyline_sfs(pts)]
    if pts.shape[0] <= 300:
        out.append(oracle_mod.skyline_pure_python(pts))
    return out


# ---------------------------------------------------------------- T1
def test_restaurants_table1(oracle_mod):
    g = _gold("restaurants.json")
    pts = np.asarray(g["points"], dtype=np.float32)
    for res in _all_impls(oracle_mod, pts):
        assert res.tolist() == g["skyline"]
    for a, b in g["dominations"]:
        assert oracle_mod.dominates(pts[a], pts[b])
        assert not oracle_mod.dominates(pts[b], pts[a])
    # the same data as uint16 (exact integers)
    for res in (oracle_mod.skyline_bruteforce(pts.astype(np.uint16)),
                oracle_mod.skyline_sfs(pts.astype(np.uint16))):
        assert res.tolist() == g["skyline"]


# ---------------------------------------------------------------- T2
def test_eq1_cell_example(oracle_mod):
    g = _gold("eq1_cell_example.json")
    dim1, dim0 = g["point_dim1_dim0"]
    p = np.asarray([[dim0, dim1]], dtype=np.float32)  # dimension order 0, 1
    for lay in g["layers"]:
        c = oracle_mod.cell_coords(p, lay["g"])[0]
        assert [int(c[1]), int(c[0])] == lay["cell_dim1_dim0"]
        assert lay["g"] == 2 ** lay["layer"]


def test_quantiser_edges(oracle_mod):
    x = np.asarray([[0.0, -0.0, 1.0, -1.0, np.inf, -np.inf, 0.999999940395, 0.5]], dtype=np.float32)
    c = oracle_mod.cell_coords(x, 8)[0].tolist()
    assert c == [0, 0, 7, 0, 7, 0, 7, 4]
    # NaN is rejected
    with pytest.raises(ValueError):
        oracle_mod.cell_coords(np.asarray([[np.nan]], dtype=np.float32), 4)
    # uint16 form: floor(v * g / 2^bits), clamped
    v = np.asarray([[0, 127, 128, 1023, 1024, 65535]], dtype=np.uint16)
    assert oracle_mod.cell_coords(v, 8, value_bits=10)[0].tolist() == [0, 0, 1, 7, 7, 7]


def test_quantiser_monotone(oracle_mod):
    rng = np.random.default_rng(3)
    x = np.sort(rng.random(5000).astype(np.float32) * 1.2 - 0.1)
    for g in (1, 2, 3, 5, 7, 8, 16):
        c = oracle_mod.cell_coords(x[:, None], g)[:, 0]
        assert np.all(np.diff(c) >= 0)
        assert c.min() >= 0 and c.max() <= g - 1


# ---------------------------------------------------------------- T3
def test_candidate_count_paper_numbers():
    g = _gold("candidate_counts.json")
    assert [C.candidate_count_closed_form(2 ** i, 2) for i in range(5)] == g["d2_layers_0_to_4"]
    assert C.candidate_count_closed_form(8, 2) == g["d2_8x8"]["count"]
    assert round(100 * g["d2_8x8"]["count"] / 64) == g["d2_8x8"]["percent_printed"]
    assert C.candidate_count_closed_form(32, 2) == g["d2_32x32"]["count"]
    assert round(100 * 63 / 1024, 1) == g["d2_32x32"]["percent_printed"]
    frac = C.candidate_count_closed_form(2 ** 10, 10) / (2 ** 10) ** 10
    assert abs(100 * frac - g["d10_rho10_percent_about"]) < 0.1


def test_candidate_count_geometric_sum():
    # Corollary 2's proof: the sum adds up to g^d - (g-1)^d
    for g in range(1, 12):
        for d in range(1, 7):
            assert C.candidate_count_closed_form(g, d) == g ** d - (g - 1) ** d


@pytest.mark.parametrize("g,d,occupancy", [(1, 2, 0.5), (2, 2, 0.5), (4, 2, 0.3), (8, 2, 0.1),
                                           (8, 2, 0.6), (3, 3, 0.2), (4, 3, 0.1), (4, 3, 0.5),
                                           (2, 4, 0.3), (5, 2, 0.0), (5, 2, 1.0)])
def test_candidate_count_bijection_brute_force(g, d, occupancy):
    """Theorem 1 / Corollary 1 by brute force: for any occupancy the number of
    candidate cells (auxiliary key cells included) is exactly Equation 14, and
    Psi maps candidates one-to-one onto the auxiliary candidate cells."""
    rng = np.random.default_rng(int(g * 100 + d * 10 + occupancy * 7))
    allc = list(itertools.product(range(g), repeat=d))
    ne = {c for c in allc if rng.random() < occupancy}
    cand = C.candidate_cells(ne, g, d)
    assert len(cand) == C.candidate_count_closed_form(g, d)
    keys = list(C.key_cells(ne, g, d)) + C.auxiliary_key_cells(g, d)
    aux = C.auxiliary_candidate_cells(g, d)
    images = {C.psi(c, keys, g) for c in cand}
    assert images == aux
    for ca in aux:
        assert C.psi(C.theta(ca, keys, g), keys, g) == ca
    # non-empty cells that are not dominated are all candidates
    dom = C.dominated_cells(ne)
    assert (ne - dom) <= cand


# ---------------------------------------------------------------- T4
def _p2m(t):
    """paper tuple [dim1, dim0] -> (dim0, dim1)"""
    return (t[1], t[0])


def test_fig1_cells():
    f = _gold("fig1_cells.json")
    g = f["g"]
    ne = {_p2m(t) for t in f["nonempty"]}
    cls = C.classify(ne, g, 2)
    assert cls[_p2m(f["dominated"]["cell"])] == "dominated"
    assert C.dominates_cell(_p2m(f["dominated"]["by"]), _p2m(f["dominated"]["cell"]))
    assert cls[_p2m(f["irrelevant"])] == "irrelevant"
    for t in f["candidate_examples"]:
        assert cls[_p2m(t)] == "candidate"
    keys = C.key_cells(ne, g, 2)
    for t in f["partial_key_cells_of_4_6"]:
        assert _p2m(t) in keys
        assert C.partially_dominates_cell(_p2m(t), _p2m([4, 6]))
    for k, v in f["omega_4_6"].items():
        assert C.omega(_p2m([4, 6]), _p2m(json.loads(k))) == v
    kw = list(keys) + C.auxiliary_key_cells(g, 2)
    assert C.big_omega(_p2m([4, 6]), kw) == f["Omega_4_6"]
    assert C.psi(_p2m([4, 6]), kw, g) == _p2m(f["Psi_4_6"])
    assert C.theta(_p2m([4, 15]), kw, g) == _p2m(f["Theta_4_15"])
    # Corollary 3 chain: the layer-4 key cells, halved layer by layer, give key cells
    for step in f["key_chain"]:
        shift = 4 - step["layer"]
        ne_l = {(a >> shift, b >> shift) for a, b in ne}
        assert _p2m(step["cell"]) in C.key_cells(ne_l, 2 ** step["layer"], 2)


def test_cells_dominated_c_vs_python(oracle_mod):
    rng = np.random.default_rng(11)
    for d in (1, 2, 3, 5):
        cells = np.unique(rng.integers(0, 5, size=(200, d)), axis=0).astype(np.int32)
        got = oracle_mod.cells_dominated(cells)
        ref = C.dominated_cells({tuple(c) for c in cells.tolist()})
        assert {tuple(c) for c, f in zip(cells.tolist(), got) if f} == ref


# ---------------------------------------------------------------- T5
def _invariants(oracle_mod, pts, sky):
    n = pts.shape[0]
    s = set(sky.tolist())
    # (i) no output point is dominated by any input point
    assert oracle_mod.is_skyline(pts, sky).all()
    # (ii) every other point is dominated by some output point
    others = np.asarray([i for i in range(n) if i not in s], dtype=np.int64)
    if others.size:
        sp = pts[sky].astype(np.float64)
        op = pts[others].astype(np.float64)
        le = (sp[None, :, :] <= op[:, None, :]).all(axis=2)
        lt = (sp[None, :, :] < op[:, None, :]).any(axis=2)
        assert (le & lt).any(axis=1).all()


@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
@pytest.mark.parametrize("d", [2, 3, 5])
def test_invariants(oracle_mod, dist, d):
    pts = datagen.generate(dist, 1500, d, seed=5)
    sky = oracle_mod.skyline_sfs(pts)
    assert np.array_equal(sky, oracle_mod.skyline_bruteforce(pts))
    _invariants(oracle_mod, pts, sky)
    rng = np.random.default_rng(1)
    # (iii) permuting points
    perm = rng.permutation(pts.shape[0])
    sky_p = oracle_mod.skyline_sfs(pts[perm])
    assert np.array_equal(np.sort(perm[sky_p]), sky)
    # (iv) permuting dimensions
    dp = rng.permutation(d)
    assert np.array_equal(oracle_mod.skyline_sfs(np.ascontiguousarray(pts[:, dp])), sky)
    # (v) strictly increasing maps per dimension (scaling by 2^k, a rank transform)
    scaled = (pts * np.float32(4.0)).astype(np.float32)
    assert np.array_equal(oracle_mod.skyline_sfs(scaled), sky)
    ranks = np.empty_like(pts)
    for k in range(d):
        ranks[:, k] = np.unique(pts[:, k], return_inverse=True)[1].astype(np.float32)
    assert np.array_equal(oracle_mod.skyline_sfs(ranks), sky)
    # (viii) merge law: sky(A u B) = sky(sky(A) u sky(B))
    half = pts.shape[0] // 2
    sa = oracle_mod.skyline_sfs(pts[:half])
    sb = oracle_mod.skyline_sfs(pts[half:]) + half
    merged = np.concatenate([sa, sb])
    sm = oracle_mod.skyline_sfs(np.ascontiguousarray(pts[merged]))
    assert np.array_equal(np.sort(merged[sm]), sky)


def test_duplicates(oracle_mod):
    rng = np.random.default_rng(2)
    base = datagen.independent(400, 3, seed=8)
    sky = oracle_mod.skyline_sfs(base)
    reps = rng.integers(1, 4, size=base.shape[0])
    dup = np.repeat(base, reps, axis=0)
    owner = np.repeat(np.arange(base.shape[0]), reps)
    sky_d = oracle_mod.skyline_sfs(dup)
    # every copy of a skyline point is output, no copy of a dominated point is
    assert np.array_equal(sky_d, np.nonzero(np.isin(owner, sky))[0])


# ---------------------------------------------------------------- T6
def _staircase_2d(pts):
    """Two-dimensional maxima by one sort and a sweep (Kung, Luccio and Preparata).

    Sorted by x0 then x1, a point is on the staircase iff it has the smallest x1
    of its x0-group and that x1 is below the x1 of every point with smaller x0."""
    x0 = pts[:, 0].astype(np.float64)
    x1 = pts[:, 1].astype(np.float64)
    order = np.lexsort((x1, x0))
    out = []
    best_before = math.inf
    i = 0
    n = len(order)
    while i < n:
        j = i
        while j < n and x0[order[j]] == x0[order[i]]:
            j += 1
        gmin = x1[order[i]]
        if gmin < best_before:
            out.extend(int(order[t]) for t in range(i, j) if x1[order[t]] == gmin)
        best_before = min(best_before, gmin)
        i = j
    return np.sort(np.asarray(out, dtype=np.int32))


@pytest.mark.parametrize("seed", range(4))
def test_2d_staircase(oracle_mod, seed):
    for pts in (datagen.anticorrelated(3000, 2, seed), datagen.small_integers(500, 2, seed, high=6),
                datagen.independent(3000, 2, seed)):
        ref = _staircase_2d(pts)
        assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)
        assert np.array_equal(oracle_mod.skyline_bruteforce(pts), ref)


def test_1d_all_minimum_copies(oracle_mod):
    pts = datagen.small_integers(300, 1, 4, high=9)
    ref = np.nonzero(pts[:, 0] == pts[:, 0].min())[0].astype(np.int32)
    assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)
    assert np.array_equal(oracle_mod.skyline_bruteforce(pts), ref)


def test_special_cases(oracle_mod):
    one = np.asarray([[0.3, 0.2, 0.9]], dtype=np.float32)
    assert oracle_mod.skyline_sfs(one).tolist() == [0]
    same = np.tile(one, (7, 1))
    assert oracle_mod.skyline_sfs(same).tolist() == list(range(7))
    pts = datagen.independent(500, 4, seed=3) + np.float32(0.01)
    pts[[17, 230]] = 0.0  # two copies of a point below everything
    assert oracle_mod.skyline_sfs(pts).tolist() == [17, 230]
    empty = np.zeros((0, 3), dtype=np.float32)
    assert oracle_mod.skyline_sfs(empty).size == 0
    assert oracle_mod.skyline_bruteforce(empty).size == 0
    with pytest.raises(ValueError):
        bad = one.copy()
        bad[0, 1] = np.nan
        oracle_mod.skyline_sfs(bad)


def test_correlated_zero_rows(oracle_mod):
    pts = datagen.correlated(20000, 4, seed=0)
    zero = np.nonzero((pts == 0).all(axis=1))[0]
    sky = oracle_mod.skyline_sfs(pts)
    if zero.size:
        assert np.array_equal(sky, zero.astype(np.int32))
    _invariants(oracle_mod, pts, sky)


# ---------------------------------------------------------------- T7
def test_exhaustive_tiny(oracle_mod):
    vals = [0.0, 1.0, 2.0]
    for d, max_pts in ((1, 5), (2, 4), (3, 3)):
        cells = list(itertools.product(vals, repeat=d))
        for m in range(1, max_pts + 1):
            for combo in itertools.combinations_with_replacement(range(len(cells)), m):
                pts = np.asarray([cells[c] for c in combo], dtype=np.float32)
                ref = oracle_mod.skyline_pure_python(pts)
                assert np.array_equal(oracle_mod.skyline_bruteforce(pts), ref)
                assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)
                assert np.array_equal(oracle_mod.skyline_kdtree(pts), ref)
                if d == 2:
                    assert np.array_equal(_staircase_2d(pts), ref)


@pytest.mark.parametrize("seed", range(3))
def test_random_ties_three_ways(oracle_mod, seed):
    for d in (2, 3, 4, 6):
        pts = datagen.small_integers(250, d, seed, high=4)
        ref = oracle_mod.skyline_pure_python(pts)
        assert np.array_equal(oracle_mod.skyline_bruteforce(pts), ref)
        assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)
        u = pts.astype(np.uint16)
        assert np.array_equal(oracle_mod.skyline_sfs(u), ref)
        assert np.array_equal(oracle_mod.skyline_bruteforce(u), ref)
        assert np.array_equal(oracle_mod.skyline_kdtree(pts), ref)
        assert np.array_equal(oracle_mod.skyline_kdtree(u), ref)


def test_sfs_matches_bruteforce_medium(oracle_mod):
    for dist in datagen.DISTRIBUTIONS:
        pts = datagen.generate(dist, 12000, 4, seed=2)
        assert np.array_equal(oracle_mod.skyline_sfs(pts), oracle_mod.skyline_bruteforce(pts))
    u = datagen.quantise_u16(datagen.anticorrelated(12000, 6, seed=1))
    assert np.array_equal(oracle_mod.skyline_sfs(u), oracle_mod.skyline_bruteforce(u))


def test_is_skyline_matches(oracle_mod):
    pts = datagen.anticorrelated(5000, 5, seed=4)
    sky = set(oracle_mod.skyline_sfs(pts).tolist())
    idx = np.arange(0, 5000, 7)
    got = oracle_mod.is_skyline(pts, idx)
    assert got.tolist() == [int(i) in sky for i in idx]


# ---------------------------------------------------------------- T8
def _expected_skyline_size(n, d):
    """Expected skyline size of n independent continuous points in d dimensions:
    A(n, 1) = 1, A(n, d) = sum_{k<=n} A(k, d-1) / k."""
    a = np.ones(n + 1)
    a[0] = 0.0
    for _ in range(2, d + 1):
        k = np.arange(n + 1, dtype=np.float64)
        k[0] = 1.0
        b = np.cumsum(a / k)
        b[0] = 0.0
        a = b
    return a[n]


def test_expected_skyline_size_plausibility(oracle_mod):
    e = _expected_skyline_size(10_000, 4)
    assert 160 < e < 170
    sizes = [oracle_mod.skyline_sfs(datagen.independent(10_000, 4, seed=s)).size for s in range(8)]
    assert abs(np.mean(sizes) - e) < 0.15 * e


# ---------------------------------------------------------------- O3 (k-d tree orthant test)
@pytest.mark.parametrize("dist", datagen.DISTRIBUTIONS)
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8, 12, 16])
def test_kdtree_matches_bruteforce(oracle_mod, dist, d):
    """O3 against the definition written out (O1) on inputs large enough for a
    deep tree (leaves of 24 points), and against the sort-first skyline (O2)."""
    pts = datagen.generate(dist, 6000 + 7 * d, d, seed=50 + d)
    ref = oracle_mod.skyline_bruteforce(pts)
    assert np.array_equal(oracle_mod.skyline_kdtree(pts), ref)
    assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)


@pytest.mark.parametrize("seed", range(4))
def test_kdtree_heavy_ties_duplicates_and_u16(oracle_mod, seed):
    """Equal coordinates, exact copies (many in one leaf, whole subtrees of one
    value) and integer data: copies never dominate each other."""
    rng = np.random.default_rng(seed)
    for d, high in ((2, 3), (4, 2), (5, 6), (7, 3)):
        base = rng.integers(0, high, size=(3000, d))
        pts = np.concatenate([base, base[:500], np.zeros((300, d), np.int64) + 1]).astype(np.float32)
        ref = oracle_mod.skyline_bruteforce(pts)
        assert np.array_equal(oracle_mod.skyline_kdtree(pts), ref)
        assert np.array_equal(oracle_mod.skyline_kdtree(pts.astype(np.uint16)), ref)
    same = np.ones((5000, 3), np.float32)
    assert np.array_equal(oracle_mod.skyline_kdtree(same), np.arange(5000, dtype=np.int32))
    u = datagen.quantise_u16(datagen.anticorrelated(20000, 6, seed=seed))
    assert np.array_equal(oracle_mod.skyline_kdtree(u), oracle_mod.skyline_bruteforce(u))


@pytest.mark.parametrize("seed", range(6))
def test_special_values_three_oracles(oracle_mod, seed):
    """Infinities of both signs (a point may hold +inf and -inf together),
    signed zeros and subnormals: O2 and O3 equal brute force."""
    rng = np.random.default_rng(seed)
    for n, d in ((400, 3), (3000, 5)):
        pts = rng.random((n, d)).astype(np.float32)
        specials = np.asarray([np.inf, -np.inf, 0.0, -0.0, 1e-45, -1e-45, 3e38, -3e38], np.float32)
        mask = rng.random((n, d)) < 0.3
        pts[mask] = specials[rng.integers(0, len(specials), size=mask.sum())]
        ref = oracle_mod.skyline_bruteforce(pts)
        assert np.array_equal(oracle_mod.skyline_sfs(pts), ref)
        assert np.array_equal(oracle_mod.skyline_kdtree(pts), ref)


def test_kdtree_matches_sfs_at_2e5(oracle_mod):
    """Larger inputs: O3 against O2 on the three distributions at d = 8, and on
    quantised data with ties."""
    for dist in datagen.DISTRIBUTIONS:
        pts = datagen.generate(dist, 200_000, 8, seed=9)
        assert np.array_equal(oracle_mod.skyline_kdtree(pts), oracle_mod.skyline_sfs(pts))
    u = datagen.quantise_u16(datagen.anticorrelated(200_000, 6, seed=9))
    assert np.array_equal(oracle_mod.skyline_kdtree(u), oracle_mod.skyline_sfs(u))


def test_kdtree_detects_a_planted_dominator(oracle_mod):
    """A single point planted just below one skyline point in every dimension
    removes it and nothing else that it does not dominate."""
    pts = datagen.anticorrelated(50_000, 6, seed=3)
    sky = oracle_mod.skyline_kdtree(pts)
    victim = int(sky[len(sky) // 2])
    planted = np.nextafter(pts[victim], np.float32(-1.0))[None, :]
    more = np.concatenate([pts, planted])
    got = oracle_mod.skyline_kdtree(more)
    assert victim not in set(got.tolist()) and 50_000 in set(got.tolist())
    assert np.array_equal(got, oracle_mod.skyline_bruteforce(more))


# ---------------------------------------------------------------- Algorithm 3
def _brute_cell_types(cells, nonempty):
    """Definitions 3-4 by brute force over explicit cells: per row,
    'dominated' (a non-empty cell is below in every dimension), 'key'
    (non-empty, no other non-empty cell <= it), else 'other'."""
    ne = [tuple(c) for c, e in zip(cells.tolist(), nonempty.tolist()) if e]
    out = []
    for c, e in zip(cells.tolist(), nonempty.tolist()):
        c = tuple(c)
        if any(C.dominates_cell(a, c) for a in ne):
            out.append("dominated")
        elif e and not any(a != c and all(x <= y for x, y in zip(a, c)) for a in ne):
            out.append("key")
        else:
            out.append("other")
    return out


def test_alg3_counterexample_two_minimal_cells():
    """Section V-B, Theorem 2 does not hold in general: with the non-empty cells
    (c0, c1) = (1,0), (0,1), (2,1) of a 3 x 3 grid, (1,0) dominates (2,1), but
    the tree's single pointer reaches (2,1) through (0,1), which only partially
    dominates it, so Algorithm 3 reports a candidate cell (Definition 3 says
    dominated).  With (1,2) in place of (2,1) the dominator is the one the tree
    keeps and the verdict is right."""
    ne = np.ones(3, bool)
    cells = np.array([(1, 0), (0, 1), (2, 1)])
    assert list(C.classify_parallel(cells, ne)) == ["key", "key", "candidate"]
    assert C.dominated_cells([(1, 0), (0, 1), (2, 1)]) == {(2, 1)}
    cells = np.array([(0, 1), (1, 0), (1, 2)])
    assert list(C.classify_parallel(cells, ne)) == ["key", "key", "dominated"]


def test_alg3_follows_the_tree_by_hand():
    """A worked run of the two sweeps on four cells in two dimensions, traced by
    hand from Algorithm 3: sorted order (dimension 1 major) (0,0) (1,0) (0,1)
    (1,1); (0,0) is the only non-empty cell and 2-dominates all others."""
    cells = np.array([(1, 1), (0, 1), (1, 0), (0, 0)])
    ne = np.array([False, False, False, True])
    o, l = C.shrink_key_cells_parallel(cells, ne)
    assert o.tolist() == [3, 2, 1, 0]          # leaves in sorted order
    assert l.tolist() == [3, 3, 3, 3]          # every l points at (0,0)
    assert list(C.classify_parallel(cells, ne)) == ["dominated", "candidate", "candidate", "key"]


@pytest.mark.parametrize("seed", range(6))
def test_alg3_verdicts_are_one_sided(seed):
    """On random occupancies (d = 2..4, every cell a leaf or only the non-empty
    ones): a 'dominated' verdict is always right (the pointer dominates the
    cell), every key cell of Definition 4 comes out as a key cell, and a
    non-empty cell is never left unclassified."""
    rng = np.random.default_rng(seed)
    for trial in range(40):
        d = int(rng.integers(2, 5))
        g = int(rng.integers(2, 6))
        allc = np.array(list(itertools.product(range(g), repeat=d)))
        occ = rng.random(len(allc)) < rng.choice([0.05, 0.2, 0.5])
        if trial % 2:
            cells, ne = allc[occ], occ[occ]
        else:
            cells, ne = allc, occ
        if cells.shape[0] == 0:
            continue
        got = C.classify_parallel(cells, ne)
        want = _brute_cell_types(cells, ne)
        for gv, wv, e in zip(got, want, ne):
            if gv == "dominated":
                assert wv == "dominated"
            if wv == "key":
                assert gv == "key"
            if e:
                assert gv != "irrelevant"


def test_alg3_exact_on_two_dimensional_chains():
    """In two dimensions (one rotation), with only non-empty cells as leaves, and
    where every cell has a single minimal non-empty cell below it (the non-empty
    cells form a chain), Theorem 2 holds: the verdicts equal the definitions.
    (Empty leaves break it even then: a subtree whose last cell is empty and
    not 2-dominated inside it passes that empty cell up as its pointer.)"""
    rng = np.random.default_rng(7)
    for trial in range(30):
        g = 7
        steps = rng.integers(0, 2, size=(g, 2))
        chain = np.unique(np.minimum(np.cumsum(steps, axis=0), g - 1), axis=0)
        allc = np.array(list(itertools.product(range(g), repeat=2)))
        ne = np.array([any((c == ch).all() for ch in chain) for c in allc])
        for cells, nn in ((allc[ne], ne[ne]),):
            got = C.classify_parallel(cells, nn)
            want = _brute_cell_types(cells, nn)
            for gv, wv in zip(got, want):
                assert (gv == "dominated") == (wv == "dominated")
                assert (gv == "key") == (wv == "key")


def test_alg3_rotations_do_not_compose_through_empty_leaves():
    """A second departure, in three dimensions: with all eight cells of a
    2 x 2 x 2 split as leaves and only (0,0,0) and (1,1,1) non-empty, each
    rotation's 2-domination test compares the pointers themselves, which never
    agree with (1,1,1) in the d - 2 dimensions the test holds fixed, so
    Algorithm 3 reports (1,1,1) as a key cell although (0,0,0) dominates it."""
    allc = np.array(list(itertools.product(range(2), repeat=3)))
    ne = np.array([tuple(c) in ((0, 0, 0), (1, 1, 1)) for c in allc.tolist()])
    got = dict(zip(map(tuple, allc.tolist()), C.classify_parallel(allc, ne)))
    assert got[(1, 1, 1)] == "key"
    assert got[(0, 0, 0)] == "key"
    assert C.dominated_cells([(0, 0, 0), (1, 1, 1)]) == {(1, 1, 1)}


def test_alg3_layers_keep_every_survivor():
    """The layer loop of Algorithm 1 with Algorithm 3: at every layer, each
    non-empty cell that Definition 3 keeps is a key or candidate cell (the
    errors of Algorithm 3 only keep extra cells)."""
    rng = np.random.default_rng(3)
    for d, rho in ((2, 4), (3, 3), (4, 2)):
        x = rng.random((300, d)).astype(np.float32)
        def layer_cells(i):
            return {tuple(c) for c in np.floor(x.astype(np.float64) * (1 << i)).astype(int).tolist()}
        res = C.layers_parallel(layer_cells, rho, d)
        for i in range(1, rho + 1):
            ne = layer_cells(i)
            surv = ne - C.dominated_cells(ne)
            kept = {c for c, t in res[i].items() if c in ne}
            assert surv <= kept, (d, i)
