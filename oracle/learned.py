"""CPU oracle for the learned pivot proposer and the pivot pre-filter.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``): only ``tests/``,
``__graft_entry__.smoke()`` and ``bench.py``'s ``cpu_baseline`` leg use it.

The proposer is not part of the paper: it is a scoring network bolted onto the
exact method, which still decides every output.  What it computes is fixed
here, in float64, step by step:

* features of a point x with g columns per dimension (2d values):
  f[k] = x[k] and f[d + k] = t - floor(t) with t = x[k] * g, both in binary32
  (the fractional position of x inside its column of Equation 1);
* a two-hidden-layer perceptron 2d -> 64 -> 64 -> 1 with ReLU and a logistic
  output; its weights are stored in bfloat16 and every matrix product takes
  bfloat16 operands (the features, the hidden activations, the back-propagated
  pre-activation gradients) with wide accumulation;
* the mean binary cross-entropy against skyline labels (1 = skyline point) and
  its gradient, passing straight through the bfloat16 roundings;
* one Adam step (Kingma and Ba, 2015) on the float32 master weights.

With ``rounding=False`` every bfloat16 rounding is skipped, which makes the
network plain float64 arithmetic: the tests pin that form against autograd and
finite differences, and the rounded form against the library's own bfloat16
conversion and closed forms.

Also here: the top-k order of scores, and the set of points the pivot
pre-filter may remove (a pivot v removes q when v dominates q, Definition 1;
the skyline is unchanged because dominance is transitive).

Flat parameter layout (float32, count = 128 d + 4289):
  W1 [64][2d] (output unit major), b1 [64], W2 [64][64] (output unit major),
  b2 [64], w3 [64], b3 [1].
"""
import numpy as np

HIDDEN = 64


def num_params(d):
    return HIDDEN * 2 * d + HIDDEN + HIDDEN * HIDDEN + HIDDEN + HIDDEN + 1


def unpack(params, d):
    """Split a flat parameter vector into (W1, b1, W2, b2, w3, b3) views."""
    p = np.asarray(params, dtype=np.float64)
    if p.shape != (num_params(d),):
        raise ValueError("expected %d parameters for d = %d" % (num_params(d), d))
    f = 2 * d
    o = 0
    W1 = p[o:o + HIDDEN * f].reshape(HIDDEN, f); o += HIDDEN * f
    b1 = p[o:o + HIDDEN]; o += HIDDEN
    W2 = p[o:o + HIDDEN * HIDDEN].reshape(HIDDEN, HIDDEN); o += HIDDEN * HIDDEN
    b2 = p[o:o + HIDDEN]; o += HIDDEN
    w3 = p[o:o + HIDDEN]; o += HIDDEN
    b3 = p[o:o + 1]
    return W1, b1, W2, b2, w3, b3


def pack(W1, b1, W2, b2, w3, b3):
    return np.concatenate([np.ravel(W1), np.ravel(b1), np.ravel(W2), np.ravel(b2),
                           np.ravel(w3), np.ravel(b3)]).astype(np.float64)


def bf16_round(x):
    """Round real values to the nearest bfloat16 value (8 significant bits, ties
    to even), from the definition of the format: same exponent range as
    binary32, 7 stored fraction bits, subnormal spacing 2^-133."""
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    nz = (x != 0) & np.isfinite(x)
    m, e = np.frexp(x[nz])           # x = m * 2^e, 0.5 <= |m| < 1
    e = np.maximum(e, -125)          # below 2^-126 the spacing stays 2^-133
    quantum = np.ldexp(1.0, e - 8)
    out[nz] = np.rint(x[nz] / quantum) * quantum   # rint: half to even
    out[~nz] = x[~nz]
    return out


def features(points, g):
    """2d features per point, computed in binary32 as the definition says,
    returned as float64 [n, 2d]."""
    x = np.asarray(points, dtype=np.float32)
    t = x * np.float32(g)            # binary32 product, round to nearest
    frac = t - np.floor(t)           # binary32 difference
    return np.concatenate([x, frac.astype(np.float32)], axis=1).astype(np.float64)


def _r(v, rounding):
    return bf16_round(v) if rounding else v


def forward(params, points, g, rounding=True):
    """Logits of the network for every point, with the intermediates."""
    n, d = np.asarray(points).shape
    W1, b1, W2, b2, w3, b3 = (_r(a, rounding) for a in unpack(params, d))
    f = _r(features(points, g), rounding)
    pre1 = f @ W1.T + b1
    h1 = _r(np.maximum(pre1, 0.0), rounding)
    pre2 = h1 @ W2.T + b2
    h2 = _r(np.maximum(pre2, 0.0), rounding)
    z = h2 @ w3 + b3[0]
    return {"f": f, "pre1": pre1, "h1": h1, "pre2": pre2, "h2": h2, "z": z,
            "W1": W1, "W2": W2, "w3": w3}


def softplus(z):
    return np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))


def sigmoid(z):
    return 0.5 * (1.0 + np.tanh(0.5 * z))


def loss_and_grad(params, points, labels, g, rounding=True):
    """Mean binary cross-entropy of sigmoid(z) against labels and its gradient
    with respect to the flat parameters (bfloat16 roundings passed straight
    through; the operands of the gradient matrix products are rounded as in the
    forward pass)."""
    n, d = np.asarray(points).shape
    y = np.asarray(labels, dtype=np.float64)
    fw = forward(params, points, g, rounding)
    z = fw["z"]
    loss = float(np.mean(softplus(z) - y * z))
    dz = sigmoid(z) - y                                  # per point, unscaled
    g_w3 = fw["h2"].T @ dz
    g_b3 = np.array([dz.sum()])
    dpre2 = np.outer(dz, fw["w3"]) * (fw["pre2"] > 0)
    dpre2_r = _r(dpre2, rounding)
    g_W2 = dpre2_r.T @ fw["h1"]
    g_b2 = dpre2.sum(axis=0)
    dh1 = dpre2_r @ fw["W2"]
    dpre1 = dh1 * (fw["pre1"] > 0)
    g_W1 = _r(dpre1, rounding).T @ fw["f"]
    g_b1 = dpre1.sum(axis=0)
    grad = pack(g_W1, g_b1, g_W2, g_b2, g_w3, g_b3) / n
    return loss, grad


def adam_step(params, grad, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam with bias correction, step number t >= 1 (Kingma and Ba, 2015,
    Algorithm 1)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    p = np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v


def topk(scores, k):
    """Indices of the k largest scores, largest first, equal scores by ascending
    index (-0.0 and +0.0 compare equal)."""
    s = np.asarray(scores, dtype=np.float32).astype(np.float64)
    if np.isnan(s).any():
        raise ValueError("scores hold NaN")
    order = np.lexsort((np.arange(s.size), -s))
    return order[:min(k, s.size)].astype(np.int32)


def dominated_by_any(points, pivots, chunk=512):
    """For every point q, whether some row v of `pivots` dominates it
    (Definition 1: v <= q in every dimension and v < q in one)."""
    q = np.asarray(points, dtype=np.float32)
    v = np.asarray(pivots, dtype=np.float32)
    out = np.zeros(q.shape[0], dtype=bool)
    if v.shape[0] == 0:
        return out
    for s in range(0, q.shape[0], chunk):
        qq = q[s:s + chunk, None, :]
        le = (v[None, :, :] <= qq).all(axis=2)
        lt = (v[None, :, :] < qq).any(axis=2)
        out[s:s + chunk] = (le & lt).any(axis=1)
    return out
