"""Pins of the learned-proposer oracle (oracle/learned.py) against things other
than itself: torch's own bfloat16 conversion and autograd, finite differences,
closed forms of special cases, and brute force for top-k and pivot removal."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import learned as L
from paper_2107_09993_amd import datagen


def rand_params(d, seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.normal(0.0, scale, L.num_params(d))


# ---------------------------------------------------------------- bfloat16
def test_bf16_round_matches_torch_conversion():
    rng = np.random.default_rng(1)
    x = np.concatenate([
        rng.normal(0, 1, 20000).astype(np.float32),
        (rng.normal(0, 1, 2000) * 1e-38).astype(np.float32),       # subnormals
        (rng.normal(0, 1, 2000) * 1e30).astype(np.float32),
        np.array([0.0, -0.0, 1.0, -1.0, 3.0, 0.1], np.float32),
    ])
    # ties: values exactly halfway between two bfloat16 neighbours
    base = rng.integers(0, 1 << 15, 2000, dtype=np.uint32) << 16 | 0x8000
    x = np.concatenate([x, base.view(np.float32)[np.isfinite(base.view(np.float32))]])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = L.bf16_round(x.astype(np.float64))
    assert np.array_equal(got, want)


def test_bf16_round_ties_to_even():
    assert L.bf16_round(np.array([1 + 2 ** -8]))[0] == 1.0
    assert L.bf16_round(np.array([1 + 3 * 2 ** -8]))[0] == 1 + 2 ** -6
    assert L.bf16_round(np.array([-(1 + 2 ** -8)]))[0] == -1.0
    assert L.bf16_round(np.array([1 + 2 ** -8 + 2 ** -30]))[0] == 1 + 2 ** -7


# ---------------------------------------------------------------- features
def test_features_known_values():
    x = np.array([[0.5, 0.0625, 1.0, 0.0]], np.float32)
    f = L.features(x, 8)
    assert f.shape == (1, 8)
    assert list(f[0, :4]) == [0.5, 0.0625, 1.0, 0.0]
    assert list(f[0, 4:]) == [0.0, 0.5, 0.0, 0.0]
    # Equation 1 example value 0.63 with g = 8: binary32 product 5.04 -> 0.04...
    t = np.float32(0.63) * np.float32(8)
    assert L.features(np.array([[0.63]], np.float32), 8)[0, 1] == float(t - np.float32(5))
    # negative values fall in [0, 1] too
    neg = L.features(np.array([[-0.3]], np.float32), 4)[0, 1]
    assert 0.0 <= neg <= 1.0


# ---------------------------------------------------------------- forward
def test_forward_zero_weights_is_output_bias():
    d = 3
    p = np.zeros(L.num_params(d))
    p[-1] = 0.75
    x = datagen.generate("independent", 50, d, 0)
    assert np.all(L.forward(p, x, 4)["z"] == 0.75)


def test_forward_selects_the_right_feature():
    """A network that routes one chosen feature to the output: a transposed
    weight matrix or a shifted feature index would route another one."""
    d = 4
    x = datagen.generate("independent", 64, d, 3)
    for feat in (0, 2, d + 1, 2 * d - 1):
        W1 = np.zeros((64, 2 * d)); W1[5, feat] = 1.0
        W2 = np.zeros((64, 64)); W2[9, 5] = 1.0
        w3 = np.zeros(64); w3[9] = 1.0
        p = L.pack(W1, np.zeros(64), W2, np.zeros(64), w3, np.zeros(1))
        z = L.forward(p, x, 8, rounding=False)["z"]
        assert np.array_equal(z, L.features(x, 8)[:, feat])


def test_forward_relu_and_biases():
    d = 1
    x = np.array([[0.25], [0.75]], np.float32)
    W1 = np.zeros((64, 2)); W1[0, 0] = 2.0
    b1 = np.zeros(64); b1[0] = -1.0              # 2x - 1: -0.5 and 0.5
    W2 = np.zeros((64, 64)); W2[1, 0] = -3.0
    b2 = np.zeros(64); b2[1] = 2.0               # 2 - 3 relu(2x - 1): 2 and 0.5
    w3 = np.zeros(64); w3[1] = 0.5
    p = L.pack(W1, b1, W2, b2, w3, np.array([0.125]))
    z = L.forward(p, x, 4)["z"]
    assert list(z) == [1.125, 0.375]


# ---------------------------------------------------------------- gradients
def _torch_loss(params, x, y, g):
    d = x.shape[1]
    f = torch.from_numpy(L.features(x, g))
    p = torch.tensor(params, dtype=torch.float64, requires_grad=True)
    o = 0
    W1 = p[o:o + 64 * 2 * d].view(64, 2 * d); o += 64 * 2 * d
    b1 = p[o:o + 64]; o += 64
    W2 = p[o:o + 4096].view(64, 64); o += 4096
    b2 = p[o:o + 64]; o += 64
    w3 = p[o:o + 64]; o += 64
    b3 = p[o]
    h = torch.relu(torch.nn.functional.linear(f, W1, b1))
    h = torch.relu(torch.nn.functional.linear(h, W2, b2))
    z = h @ w3 + b3
    loss = torch.nn.functional.binary_cross_entropy_with_logits(z, torch.from_numpy(y).double())
    loss.backward()
    return loss.item(), p.grad.numpy()


@pytest.mark.parametrize("d", [1, 4, 10])
def test_gradient_unrounded_matches_autograd(d):
    x = datagen.generate("anticorrelated", 300, d, d)
    y = (np.random.default_rng(d).random(300) < 0.4).astype(np.float64)
    p = rand_params(d, d)
    loss, grad = L.loss_and_grad(p, x, y, 4, rounding=False)
    tl, tg = _torch_loss(p, x, y, 4)
    assert abs(loss - tl) <= 1e-12 * max(1.0, abs(tl))
    np.testing.assert_allclose(grad, tg, rtol=1e-9, atol=1e-13)


def test_gradient_unrounded_matches_finite_differences():
    d = 3
    x = datagen.generate("independent", 200, d, 7)
    y = (np.random.default_rng(7).random(200) < 0.5).astype(np.float64)
    p = rand_params(d, 7)
    _, grad = L.loss_and_grad(p, x, y, 8, rounding=False)
    rng = np.random.default_rng(11)
    coords = np.concatenate([rng.choice(L.num_params(d), 60, replace=False),
                             [L.num_params(d) - 1, L.num_params(d) - 2]])
    h = 1e-6
    for c in coords:
        e = np.zeros_like(p); e[c] = h
        lp, _ = L.loss_and_grad(p + e, x, y, 8, rounding=False)
        lm, _ = L.loss_and_grad(p - e, x, y, 8, rounding=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - grad[c]) <= 1e-6 * max(1e-3, abs(grad[c])) + 1e-9, c


def test_gradient_closed_form_output_bias_only():
    d = 5
    x = datagen.generate("correlated", 100, d, 1)
    y = (np.arange(100) % 3 == 0).astype(np.float64)
    p = np.zeros(L.num_params(d)); p[-1] = -0.375   # exact in bfloat16
    loss, grad = L.loss_and_grad(p, x, y, 2)
    c = -0.375
    assert math.isclose(loss, math.log1p(math.exp(c)) - y.mean() * c, rel_tol=1e-14)
    assert math.isclose(grad[-1], 1 / (1 + math.exp(-c)) - y.mean(), rel_tol=1e-12)
    assert np.all(grad[:-1] == 0.0)


def test_gradient_rounded_is_close_to_unrounded():
    """The bfloat16 roundings move the gradient by about their relative size
    (2^-8), not more: a dropped term or a wrong operand would not."""
    d = 10
    x = datagen.generate("anticorrelated", 2000, d, 5)
    y = (np.random.default_rng(5).random(2000) < 0.7).astype(np.float64)
    p = rand_params(d, 5)
    _, g0 = L.loss_and_grad(p, x, y, 4, rounding=False)
    _, g1 = L.loss_and_grad(p, x, y, 4, rounding=True)
    assert np.linalg.norm(g1 - g0) <= 0.05 * np.linalg.norm(g0)
    # and the output-bias gradient is the closed form on the rounded logits
    z = L.forward(p, x, 4)["z"]
    assert math.isclose(g1[-1], float(np.mean(1 / (1 + np.exp(-z)) - y)), rel_tol=1e-12)


# ---------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    p0 = np.array([1.0, 1.0, 1.0, 1.0])
    p, m, v = L.adam_step(p0, g, np.zeros(4), np.zeros(4), 1, 0.01)
    want = p0 - 0.01 * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(p, want, rtol=0, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_keeps_unit_steps():
    p = np.zeros(2)
    m = np.zeros(2); v = np.zeros(2)
    for t in range(1, 30):
        p, m, v = L.adam_step(p, np.array([3.0, -0.25]), m, v, t, 0.1)
    np.testing.assert_allclose(p, [-2.9, 2.9], rtol=1e-6)


# ---------------------------------------------------------------- top-k
def test_topk_brute_force_with_ties():
    rng = np.random.default_rng(2)
    for trial in range(50):
        n = int(rng.integers(1, 60))
        s = rng.integers(-3, 4, n).astype(np.float32)
        s[rng.random(n) < 0.2] = -0.0
        k = int(rng.integers(1, n + 3))
        want = sorted(range(n), key=lambda i: (-float(s[i]), i))[:k]
        assert list(L.topk(s, k)) == want


def test_topk_rejects_nan():
    with pytest.raises(ValueError):
        L.topk(np.array([1.0, np.nan], np.float32), 1)


# ---------------------------------------------------------------- pivots
def test_dominated_by_any_brute_force(oracle_mod):
    rng = np.random.default_rng(4)
    for trial in range(20):
        d = int(rng.integers(1, 5))
        x = rng.integers(0, 4, (40, d)).astype(np.float32)
        piv = x[rng.choice(40, 7, replace=False)]
        got = L.dominated_by_any(x, piv)
        want = [any(oracle.dominates(v, q) for v in piv) for q in x]
        assert list(got) == want


def test_all_points_as_pivots_remove_exactly_the_non_skyline(oracle_mod):
    x = datagen.generate("anticorrelated", 3000, 4, 9)
    sky = oracle.skyline_bruteforce(x)
    removed = L.dominated_by_any(x, x)
    mask = np.ones(3000, bool); mask[sky] = False
    assert np.array_equal(removed, mask)
