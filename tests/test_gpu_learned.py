"""GPU parity of the learned pivot proposer against the CPU oracle.

Forward logits, loss, gradients and Adam steps of the hand-written MFMA kernels
are compared with oracle/learned.py (float64 with the same bfloat16 rounding
points).  Tolerances follow from the arithmetic: the kernels accumulate in
float32 (relative error about K * 2^-24 per sum of K terms) and a bfloat16
rounding decision (8 significant bits) can only differ from the oracle's when a
value lies that close to a rounding boundary; each such flip moves one
activation by one bfloat16 unit in the last place (at most 2^-7 of its value).
The bound used for a logit is that every hidden activation flipped at once.

Top-k and the pivot pre-filter are integer work and must match exactly; the
pivoted skyline must equal the oracle's skyline bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import learned as L
import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def soa(x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float32).T)).to(DEV)


def rand_params(d, seed, scale=0.25):
    rng = np.random.default_rng(seed)
    p = rng.normal(0.0, scale, L.num_params(d))
    return p.astype(np.float32)


def logit_bound(params, x, g):
    """Largest logit change if every hidden activation moved by 2^-7 of itself."""
    fw = L.forward(params.astype(np.float64), x, g)
    w3 = np.abs(fw["w3"])
    s2 = np.abs(fw["h2"]) @ w3
    sens1 = np.abs(fw["W2"]).T @ w3          # |dz/dh1| upper bound per unit
    s1 = np.abs(fw["h1"]) @ sens1
    return 2.0 ** -7 * (s1 + s2), fw["z"]


# ---------------------------------------------------------------- forward
@pytest.mark.parametrize("d,n,g", [(1, 37, 4), (3, 1000, 8), (8, 4099, 4), (10, 20011, 4), (16, 3001, 2)])
def test_forward_matches_oracle(d, n, g):
    x = datagen.generate("anticorrelated", n, d, 100 + d)
    p = rand_params(d, d)
    m = sky.MLP(d, g)
    m.set_params(p)
    z = m.score(soa(x)).cpu().numpy().astype(np.float64)
    bound, zo = logit_bound(p, x, g)
    err = np.abs(z - zo)
    assert np.all(err <= bound + 1e-5 * (1 + np.abs(zo))), float(np.max(err - bound))
    assert np.quantile(err / (1 + np.abs(zo)), 0.9) <= 1e-4
    m.close()


def test_forward_on_a_minibatch_slice():
    d, n = 6, 5000
    x = datagen.generate("independent", n, d, 5)
    p = rand_params(d, 9)
    m = sky.MLP(d, 8)
    m.set_params(p)
    full = soa(x)
    part = m.score(full[:, 1234:3456]).cpu().numpy()
    whole = m.score(full).cpu().numpy()
    assert np.array_equal(part, whole[1234:3456])
    m.close()


# ---------------------------------------------------------------- backward
def grad_blocks(d):
    b1 = 64 * 2 * d
    return {"W1": slice(0, b1), "b1": slice(b1, b1 + 64), "W2": slice(b1 + 64, b1 + 64 + 4096),
            "b2": slice(b1 + 4160, b1 + 4224), "w3": slice(b1 + 4224, b1 + 4288),
            "b3": slice(b1 + 4288, b1 + 4289)}


def grad_bound(params, x, y, g):
    """Element-wise bound on |kernel gradient - oracle gradient|, propagated
    through the network with absolute values.  Every bfloat16 rounding the
    kernels take (features, hidden activations, the back-propagated
    pre-activation gradients) may land one unit in the last place away from the
    oracle's (at most 2^-7 of the value); float32 sums of K terms are off by at
    most K * 2^-24 of their absolute sum; a ReLU whose pre-activation lies within
    its own error bound of zero may switch, which moves its term by its whole
    size.  Returns the flat bound in the parameter layout."""
    eps = 2.0 ** -7
    n, d = x.shape
    fw = L.forward(params.astype(np.float64), x, g)
    W1a, W2a, w3a = np.abs(fw["W1"]), np.abs(fw["W2"]), np.abs(fw["w3"])
    _, b1, _, b2, _, b3 = (np.abs(L.bf16_round(a)) for a in L.unpack(params.astype(np.float64), d))
    af, ah1, ah2 = np.abs(fw["f"]), np.abs(fw["h1"]), np.abs(fw["h2"])
    a1, a2, a3 = (2 * d + 1) * 2.0 ** -24, 65 * 2.0 ** -24, 65 * 2.0 ** -24
    an = (n + 64) * 2.0 ** -24                                   # sums over the points
    # forward
    df = eps * af
    dpre1 = df @ W1a.T + a1 * (af @ W1a.T + b1)
    dh1 = dpre1 + eps * ah1
    dpre2 = dh1 @ W2a.T + a2 * (ah1 @ W2a.T + b2)
    dh2 = dpre2 + eps * ah2
    dz = dh2 @ w3a + a3 * (ah2 @ w3a + b3[0])
    s = L.sigmoid(fw["z"]) - np.asarray(y, np.float64)
    as_, ds = np.abs(s), dz / 4.0 + 1e-7                          # sigmoid' <= 1/4
    # second layer's pre-activation gradient t2 = s * w3 (where pre2 > 0), rounded
    on2 = fw["pre2"] > 0
    flip2 = np.abs(fw["pre2"]) <= dpre2
    at2 = as_[:, None] * w3a[None, :] * on2
    dt2 = ds[:, None] * w3a[None, :] * (on2 | flip2) + as_[:, None] * w3a[None, :] * flip2 + eps * at2
    # first layer's t1 = (t2 W2) (where pre1 > 0), rounded
    ag1 = (at2 + dt2) @ W2a
    dg1 = dt2 @ W2a + a2 * ag1
    on1 = fw["pre1"] > 0
    flip1 = np.abs(fw["pre1"]) <= dpre1
    at1 = np.abs(at2 @ W2a) * on1
    dt1 = dg1 * (on1 | flip1) + ag1 * flip1 + eps * (at1 + dg1)
    # products summed over the points, plus the float32 error of those sums
    def prod(da, a, db, b):
        return (da.T @ (b + db) + a.T @ db + an * ((a + da).T @ (b + db))) / n
    bW1 = prod(dt1, at1, df, af)
    bb1 = (dt1.sum(0) + an * (at1 + dt1).sum(0)) / n
    bW2 = prod(dt2, at2, dh1, ah1)
    bb2 = (dt2.sum(0) + an * (at2 + dt2).sum(0)) / n
    bw3 = prod(ds[:, None], as_[:, None], dh2, ah2).ravel()
    bb3 = np.array([(ds.sum() + an * (as_ + ds).sum()) / n])
    return L.pack(bW1, bb1, bW2, bb2, bw3, bb3)


@pytest.mark.parametrize("d,n,g", [(2, 777, 4), (10, 8192 + 13, 4), (16, 3000, 2)])
def test_backward_matches_oracle(d, n, g):
    x = datagen.generate("anticorrelated", n, d, 7 + d)
    y = (np.random.default_rng(d).random(n) < 0.6).astype(np.uint8)
    p = rand_params(d, 3 * d)
    m = sky.MLP(d, g)
    m.set_params(p)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    m.backward(soa(x), torch.from_numpy(y).to(DEV), loss_out=loss)
    g_gpu = m.get_grads().astype(np.float64)
    lo, g_or = L.loss_and_grad(p.astype(np.float64), x, y, g)
    assert abs(float(loss.item()) - lo) <= 1e-4 * max(1.0, abs(lo))
    bound = grad_bound(p, x, y, g)
    for name, sl in grad_blocks(d).items():
        a, b, lim = g_gpu[sl], g_or[sl], bound[sl]
        err = np.abs(a - b)
        # every element within its own worst-case bound ...
        assert np.all(err <= lim), (name, int(np.argmax(err - lim)), float(np.max(err - lim)))
        # ... and the block as a whole close to the oracle's: a systematic error
        # (a scaled block, a sign, a permuted order) moves its norm
        assert np.linalg.norm(err) <= 5e-3 * max(np.linalg.norm(b), 1e-12), name
    m.close()


def test_backward_all_padding_tail_and_single_point():
    d, g = 4, 4
    x = datagen.generate("correlated", 1, d, 1)
    y = np.array([1], np.uint8)
    p = rand_params(d, 1)
    m = sky.MLP(d, g)
    m.set_params(p)
    m.backward(soa(x), torch.from_numpy(y).to(DEV))
    lo, g_or = L.loss_and_grad(p.astype(np.float64), x, y, g)
    g_gpu = m.get_grads().astype(np.float64)
    assert np.linalg.norm(g_gpu - g_or) <= 5e-3 * np.linalg.norm(g_or)
    m.close()


# ---------------------------------------------------------------- Adam
def test_adam_matches_oracle():
    d = 5
    p = rand_params(d, 4)
    rng = np.random.default_rng(8)
    m = sky.MLP(d, 4)
    m.set_params(p)
    pm, m1, m2 = p.astype(np.float64), np.zeros(L.num_params(d)), np.zeros(L.num_params(d))
    for t in range(1, 4):
        gr = (rng.normal(0, 1e-2, L.num_params(d)) * (rng.random(L.num_params(d)) < 0.9)).astype(np.float32)
        m.set_grads(gr)
        m.adam_step(0.01)
        pm, m1, m2 = L.adam_step(pm, gr.astype(np.float64), m1, m2, t, 0.01)
        got = m.get_params().astype(np.float64)
        np.testing.assert_allclose(got, pm, rtol=2e-6, atol=2e-7)
    m.close()


def test_save_load_roundtrip(tmp_path):
    d, g = 7, 8
    m = sky.MLP(d, g, seed=123)
    x = soa(datagen.generate("independent", 3000, d, 2))
    y = torch.ones(3000, dtype=torch.uint8, device=DEV)
    m.train_step(x, y, 1e-3)
    path = str(tmp_path / "net.bin")
    m.save(path)
    m2 = sky.MLP.load(path)
    assert (m2.d, m2.grid_res) == (d, g)
    assert np.array_equal(m.get_params(), m2.get_params())
    assert torch.equal(m.score(x), m2.score(x))
    # the Adam state came along: one more step moves both alike (the gradient
    # sums use float atomics, so only up to their rounding)
    m.train_step(x, y, 1e-3)
    m2.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    np.testing.assert_allclose(m.get_params(), m2.get_params(), rtol=1e-5, atol=1e-6)
    m.close()
    m2.close()


def test_create_is_seeded_and_glorot_bounded():
    d = 10
    a = sky.MLP(d, 4, seed=5).get_params()
    b = sky.MLP(d, 4, seed=5).get_params()
    c = sky.MLP(d, 4, seed=6).get_params()
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    blk = grad_blocks(d)
    lim1 = np.sqrt(6.0 / (2 * d + 64))
    assert np.all(np.abs(a[blk["W1"]]) <= lim1) and np.abs(a[blk["W1"]]).max() > 0.9 * lim1
    assert np.all(a[blk["b1"]] == 0) and np.all(a[blk["b2"]] == 0) and a[blk["b3"]][0] == 0


def test_training_lowers_the_loss():
    d, n = 6, 100_000
    x = datagen.generate("anticorrelated", n, d, 31)
    xs = soa(x)
    idx = sky.compute(xs, layout="dn")
    cnt = torch.tensor([idx.numel()], dtype=torch.int32, device=DEV)
    y = sky.skyline_labels(idx, cnt, n)
    assert int(y.sum().item()) == idx.numel()
    m = sky.MLP(d, sky.choose_grid(n, d), seed=1)
    loss = torch.zeros(1, dtype=torch.float32, device=DEV)
    m.backward(xs, y, loss_out=loss)
    first = float(loss.item())
    for epoch in range(30):
        for a in range(0, n, 16384):
            m.train_step(xs[:, a:a + 16384], y[a:a + 16384], 3e-3)
    m.backward(xs, y, loss_out=loss)
    last = float(loss.item())
    assert last < 0.9 * first, (first, last)
    m.close()


# ---------------------------------------------------------------- labels
def test_skyline_labels():
    n = 1000
    idx = torch.tensor([3, 7, 999, 0], dtype=torch.int32, device=DEV)
    cnt = torch.tensor([3], dtype=torch.int32, device=DEV)
    y = sky.skyline_labels(idx, cnt, n).cpu().numpy()
    want = np.zeros(n, np.uint8); want[[3, 7, 999]] = 1
    assert np.array_equal(y, want)
    neg = torch.tensor([-6], dtype=torch.int32, device=DEV)
    assert int(sky.skyline_labels(idx, neg, n).sum().item()) == 0


# ---------------------------------------------------------------- top-k
TOPK_CASES = [
    ("single", 1, 1), ("k_above_n", 10, 4096), ("ties_small", 5000, 100),
    ("random_mid", 100_003, 4096), ("few_values_big", 2_000_000, 4096),
    ("all_equal", 50_000, 4096), ("signed_zeros", 30_000, 777), ("k_is_n", 4096, 4096),
]


@pytest.mark.parametrize("name,n,k", TOPK_CASES, ids=[c[0] for c in TOPK_CASES])
def test_topk_matches_oracle(name, n, k):
    rng = np.random.default_rng(n + k)
    if name in ("ties_small", "few_values_big"):
        s = rng.integers(-20, 20, n).astype(np.float32) / 4
    elif name == "all_equal":
        s = np.full(n, 0.5, np.float32)
    elif name == "signed_zeros":
        s = np.where(rng.random(n) < 0.5, np.float32(-0.0), np.float32(0.0))
        s[rng.random(n) < 0.01] = 1.0
    else:
        s = rng.normal(0, 3, n).astype(np.float32)
    got = sky.topk(torch.from_numpy(s).to(DEV), k).cpu().numpy()
    assert np.array_equal(got, L.topk(s, k))


# ---------------------------------------------------------------- pivot pre-filter
def surviving_mask(x, g):
    """Definition 3 per point (oracle): the point's cell is not dominated."""
    c = oracle.cell_coords(x, g)
    cells, inv = np.unique(c, axis=0, return_inverse=True)
    dom = oracle.cells_dominated(cells.astype(np.int32))
    return ~dom[inv.reshape(-1)]


PIVOT_CASES = [
    ("anti_d4", "anticorrelated", 20000, 4, 8, "l1", 4096),
    ("ind_d8", "independent", 30000, 8, 4, "random", 1000),
    ("corr_d3", "correlated", 25000, 3, 16, "l1", 64),
    ("anti_d10", "anticorrelated", 40000, 10, 2, "l1", 4096),
    ("ties_d5", "small_integers", 20000, 5, 4, "random", 300),
    ("k_above_n", "independent", 500, 3, 4, "l1", 4096),
]


@pytest.mark.parametrize("name,dist,n,d,g,how,k", PIVOT_CASES, ids=[c[0] for c in PIVOT_CASES])
def test_compute_with_pivots(oracle_mod, name, dist, n, d, g, how, k):
    if dist == "small_integers":
        x = datagen.small_integers(n, d, seed=3, high=6)
    else:
        x = datagen.generate(dist, n, d, 40 + d)
    rng = np.random.default_rng(n)
    if how == "l1":   # pivots: smallest coordinate sums first (oracle-side choice)
        piv = L.topk(-x.astype(np.float64).sum(axis=1).astype(np.float32), k)
    else:
        piv = rng.choice(n, min(k, n), replace=False).astype(np.int32)
    want = oracle.skyline_sfs(x)
    # gated (the default): the skyline is the oracle's whatever the gate decides
    got, st = sky.compute_with_pivots(soa(x), torch.from_numpy(piv).to(DEV), grid_res=g, return_stats=True)
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["pivot_removed"] <= n - want.size
    # gate off: exactly the points of surviving cells that a pivot dominates
    # (Definition 1) are removed
    kk = min(k, n)
    surv = surviving_mask(x, g)
    removed = surv & L.dominated_by_any(x, x[piv[:kk]])
    sky.set_pivot_gate(False)
    try:
        got, st = sky.compute_with_pivots(soa(x), torch.from_numpy(piv).to(DEV), grid_res=g, return_stats=True)
    finally:
        sky.set_pivot_gate(True)
    assert np.array_equal(got.cpu().numpy(), want)
    assert st["pivot_removed"] == int(removed.sum())
    assert st["survivor_points"] == int(surv.sum()) - int(removed.sum())


def test_pivot_index_out_of_range_is_reported():
    x = soa(datagen.generate("independent", 1000, 3, 1))
    with pytest.raises(sky.SkycellError):
        sky.compute_with_pivots(x, torch.tensor([5, 1000], dtype=torch.int32, device=DEV), grid_res=4)
    with pytest.raises(sky.SkycellError):
        sky.compute_with_pivots(x, torch.tensor([-1], dtype=torch.int32, device=DEV), grid_res=4)
    # and the library keeps working afterwards
    idx = sky.compute_with_pivots(x, torch.tensor([5], dtype=torch.int32, device=DEV), grid_res=4)
    assert np.array_equal(idx.cpu().numpy(), sky.compute(x, layout="dn", grid_res=4).cpu().numpy())


@pytest.mark.parametrize("k", [1, 100, 4096])
def test_compute_pivoted_equals_oracle(oracle_mod, k):
    d, n = 8, 60000
    x = datagen.generate("anticorrelated", n, d, 77)
    m = sky.MLP(d, 4, seed=k)
    got, st = sky.compute_pivoted(soa(x), m, k=k, return_stats=True)
    assert np.array_equal(got.cpu().numpy(), oracle.skyline_sfs(x))
    assert st["skyline"] == got.numel()
    m.close()


def test_pivoted_headline_size_sampled(oracle_mod):
    """n = 2e7, d = 10 anti-correlated (the learned workload): pivoted equals
    plain exactly; sampled indices are checked against the oracle."""
    d, n = 10, 20_000_000
    x = datagen.generate("anticorrelated", n, d, 0)
    xs = soa(x)
    m = sky.MLP(d, 4, seed=0)
    piv = sky.compute_pivoted(xs, m, k=4096)
    plain = sky.compute(xs, layout="dn")
    assert torch.equal(piv, plain)
    rng = np.random.default_rng(0)
    sample = np.sort(rng.choice(n, 48, replace=False)).astype(np.int32)
    res = oracle.is_skyline(x, sample)
    got = np.isin(sample, piv.cpu().numpy())
    assert np.array_equal(got, res)
    m.close()


@pytest.mark.parametrize("dist,n", [("independent", 2_000_000), ("anticorrelated", 2_000_000)])
def test_shipped_networks_against_plain_and_smallest_sum(oracle_mod, dist, n):
    """The committed networks on their own distribution (d = 10): the pivoted
    skyline equals the oracle's and the plain path's, and what the network's
    pivots remove is reported next to the smallest-coordinate-sum pivots (a
    rule that needs no training).  On independent data the gate opens and the
    network removes most surviving points; it does not beat the sum rule."""
    from paper_2107_09993_amd import learned
    x = datagen.generate(dist, n, 10, 123)
    net = sky.MLP.load(learned.NETS[dist])
    res = learned.evaluate(net, n=n, d=10, k=4096, reps=2, device=DEV, x=x, dist=dist)
    net.close()
    assert res["identical_outputs"]
    want = oracle_mod.skyline_kdtree(x)
    assert res["skyline"] == want.size
    got = sky.compute_pivoted(soa(x), sky.MLP.load(learned.NETS[dist]), k=4096).cpu().numpy()
    assert np.array_equal(got, want)
    print("\n%s n=%d: plain %.1f ms; network pivots %.1f ms (%.2fx, %d removed); smallest-sum pivots %.1f ms "
          "(%.2fx, %d removed); random pivots %.2fx"
          % (dist, n, res["plain"]["ms"], res["learned"]["ms"], res["learned"]["speedup_vs_plain"],
             res["learned"]["pivot_removed"], res["l1_pivots"]["ms"], res["l1_pivots"]["speedup_vs_plain"],
             res["l1_pivots"]["pivot_removed"], res["random_pivots"]["speedup_vs_plain"]))
    if dist == "independent":
        # the gate opens: the network's pivots remove most surviving points
        assert res["learned"]["pivot_removed"] > 0.5 * res["plain"]["survivor_points"]
