"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no skyline arithmetic: it only draws numbers.  It stands in for
the data of the paper's experiments (Section VII-A): the commonly used
independent / correlated / anti-correlated generator and the OpenStreetMap set,
neither of which is available here.

All draws use ``numpy.random.default_rng(seed)`` (PCG64) in float64, cast to
float32 last.  Arrays are row-major ``[n, d]``.

* independent:      x_k ~ U[0, 1)  (drawn directly as float32, so always < 1)
* correlated:       t ~ U(0, 1); x_k = clip(t + N(0, 0.05), 0, 1)
* anti-correlated:  y uniform on the plane sum(y) = d/2 inside the unit cube
                    (y_1..y_{d-1} ~ U(0,1), y_d = d/2 - sum, rejected unless
                    y_d in [0, 1]); x = clip(y + N(0, 0.05) * 1/sqrt(d), 0, 1),
                    i.e. a normal offset of standard deviation 0.05 along the
                    plane's unit normal.
* quantised:        v = min(1023, floor(x * 1024)) as uint16 (values in 0..1023),
                    so equal coordinates and duplicate points are frequent.
"""
import math

import numpy as np

DISTRIBUTIONS = ("independent", "correlated", "anticorrelated")


def independent(n, d, seed):
    rng = np.random.default_rng(seed)
    return rng.random((n, d), dtype=np.float32)


def correlated(n, d, seed, sigma=0.05):
    rng = np.random.default_rng(seed)
    t = rng.random((n, 1))
    x = t + rng.normal(0.0, sigma, size=(n, d))
    return np.clip(x, 0.0, 1.0).astype(np.float32)


def _plane_points(rng, n, d):
    """Uniform points on {y in [0,1]^d : sum(y) = d/2} by rejection."""
    out = np.empty((n, d), dtype=np.float64)
    filled = 0
    while filled < n:
        need = n - filled
        batch = max(1024, int(need * 2.4) + 64)
        y = rng.random((batch, d - 1)) if d > 1 else np.empty((batch, 0))
        last = d / 2.0 - y.sum(axis=1)
        ok = (last >= 0.0) & (last <= 1.0)
        y = np.concatenate([y[ok], last[ok, None]], axis=1)
        take = min(need, y.shape[0])
        out[filled:filled + take] = y[:take]
        filled += take
    return out


def anticorrelated(n, d, seed, sigma=0.05):
    rng = np.random.default_rng(seed)
    y = _plane_points(rng, n, d)
    e = rng.normal(0.0, sigma, size=(n, 1)) / math.sqrt(d)
    return np.clip(y + e, 0.0, 1.0).astype(np.float32)


def generate(dist, n, d, seed):
    if dist in ("independent", "ind"):
        return independent(n, d, seed)
    if dist in ("correlated", "corr"):
        return correlated(n, d, seed)
    if dist in ("anticorrelated", "anti"):
        return anticorrelated(n, d, seed)
    raise ValueError("unknown distribution %r" % (dist,))


def quantise_u16(x, levels=1024):
    """Map float data in [0, 1] to integers 0..levels-1 (uint16)."""
    v = np.floor(np.asarray(x, dtype=np.float64) * levels)
    return np.minimum(v, levels - 1).astype(np.uint16)


def small_integers(n, d, seed, high=4):
    """Heavy ties: integer-valued float32 coordinates in 0..high-1."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, high, size=(n, d)).astype(np.float32)


def batched_instances(count=4096, seed=0, n_lo=1_000, n_hi=200_000, d_lo=3, d_hi=12):
    """Instance shapes of the batched workload: n log-uniform in [n_lo, n_hi],
    d uniform in {d_lo..d_hi}, distribution uniform over the three kinds.
    Instance b's data seed is 10**6 + b.  Returns a list of (n, d, dist, seed)."""
    rng = np.random.default_rng(seed)
    ns = np.floor(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), size=count))).astype(np.int64)
    ds = rng.integers(d_lo, d_hi + 1, size=count)
    kinds = rng.integers(0, 3, size=count)
    return [(int(ns[b]), int(ds[b]), DISTRIBUTIONS[int(kinds[b])], 10 ** 6 + b) for b in range(count)]
