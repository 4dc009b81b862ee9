"""Training and evaluation driver of the learned pivot proposer.

Training data: anti-correlated datasets (n points, d attributes, seeds
100, 101, ...), labelled by the plain skyline path itself (1 = skyline point);
the network is trained with the library's own forward/backward kernels and
Adam, one mini-batch after another.  Evaluation: the pivoted skyline against
the plain one on a larger anti-correlated input, with the network's top-k
points, random points and the smallest-coordinate-sum points as pivots.

    python -m paper_2107_09993_amd.learned train --dist anticorrelated   # -> nets/anti_d10.bin
    python -m paper_2107_09993_amd.learned eval --dist anticorrelated --n 20000000
    python -m paper_2107_09993_amd.learned train --dist independent      # -> nets/indep_d10.bin
    python -m paper_2107_09993_amd.learned eval --dist independent --n 5000000
"""
import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_NET = os.path.join(HERE, "nets", "anti_d10.bin")
# one trained network per training distribution
NETS = {"anticorrelated": DEFAULT_NET, "independent": os.path.join(HERE, "nets", "indep_d10.bin")}


def _soa(x, dev):
    import numpy as np
    import torch
    return torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)


def train(d=10, n=1_000_000, datasets=64, first_seed=100, epochs=2, batch=65536, lr=2e-3,
          feat_grid=4, seed=0, device="cuda", log=None, dist="anticorrelated"):
    """Train a fresh network; returns (mlp, summary dict)."""
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    dev = torch.device(device)
    mlp = sky.MLP(d, feat_grid, seed=seed)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    losses = []
    t_train = 0.0
    points_trained = 0
    for s in range(first_seed, first_seed + datasets):
        x = datagen.generate(dist, n, d, s)
        xs = _soa(x, dev)
        idx = sky.compute(xs, layout="dn")
        cnt = torch.tensor([idx.numel()], dtype=torch.int32, device=dev)
        y = sky.skyline_labels(idx, cnt, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(epochs):
            for a in range(0, n, batch):
                b = min(n, a + batch)
                mlp.train_step(xs[:, a:b], y[a:b], lr, loss_out=loss)
                points_trained += b - a
        torch.cuda.synchronize()
        t_train += time.perf_counter() - t0
        mlp.backward(xs, y, loss_out=loss)
        losses.append(float(loss.item()))
        if log:
            log(json.dumps({"dataset_seed": s, "skyline_fraction": idx.numel() / n, "loss": losses[-1]}))
    return mlp, {"distribution": dist, "datasets": datasets, "n": n, "d": d, "epochs": epochs,
                 "batch": batch, "lr": lr,
                 "feature_grid": feat_grid, "final_loss": losses[-1] if losses else None,
                 "first_loss": losses[0] if losses else None,
                 "train_points_per_s": points_trained / t_train if t_train > 0 else None}


def evaluate(mlp, n=20_000_000, d=10, seed=0, k=4096, reps=3, device="cuda", x=None, log=None,
             dist="anticorrelated"):
    """Plain vs pivoted skyline timings and counters on one input of `dist`."""
    import numpy as np
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    dev = torch.device(device)
    if x is None:
        x = datagen.generate(dist, n, d, seed)
    xs = _soa(x, dev)
    g = sky.choose_grid(n, d)

    def timed(fn):
        out = fn()  # warm-up (and the result)
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        return out, best * 1e3

    (plain, st_plain), ms_plain = timed(lambda: sky.compute(xs, layout="dn", grid_res=g, return_stats=True))
    (learned, st_l), ms_l = timed(lambda: sky.compute_pivoted(xs, mlp, k=k, grid_res=g, return_stats=True))
    rng = np.random.default_rng(seed + 1)
    rand_piv = torch.from_numpy(rng.choice(n, k, replace=False).astype(np.int32)).to(dev)
    (rnd, st_r), ms_r = timed(lambda: sky.compute_with_pivots(xs, rand_piv, grid_res=g, return_stats=True))
    l1_piv = sky.topk(-xs.sum(dim=0), k)
    (l1, st_1), ms_1 = timed(lambda: sky.compute_with_pivots(xs, l1_piv, grid_res=g, return_stats=True))
    same = bool(torch.equal(plain, learned) and torch.equal(plain, rnd) and torch.equal(plain, l1))

    def row(ms, st):
        return {"ms": ms, "pivot_removed": st["pivot_removed"], "survivor_points": st["survivor_points"],
                "pair_tests": st["pair_tests"], "speedup_vs_plain": ms_plain / ms}

    res = {"distribution": dist, "n": n, "d": d, "seed": seed, "grid_res": g, "k": k,
           "skyline": int(plain.numel()),
           "identical_outputs": same,
           "plain": {"ms": ms_plain, "survivor_points": st_plain["survivor_points"],
                     "pair_tests": st_plain["pair_tests"]},
           "learned": row(ms_l, st_l), "random_pivots": row(ms_r, st_r), "l1_pivots": row(ms_1, st_1)}
    if log:
        log(json.dumps(res))
    return res


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--out", default=None)
    t.add_argument("--dist", default="anticorrelated", choices=sorted(NETS))
    t.add_argument("--datasets", type=int, default=64)
    t.add_argument("--n", type=int, default=1_000_000)
    t.add_argument("--d", type=int, default=10)
    t.add_argument("--epochs", type=int, default=2)
    t.add_argument("--lr", type=float, default=2e-3)
    t.add_argument("--feature-grid", type=int, default=4)
    e = sub.add_parser("eval")
    e.add_argument("--net", default=None)
    e.add_argument("--dist", default="anticorrelated", choices=sorted(NETS))
    e.add_argument("--n", type=int, default=20_000_000)
    e.add_argument("--k", type=int, default=4096)
    a = ap.parse_args()
    import paper_2107_09993_amd as sky
    log = lambda s: print(s, flush=True)
    if a.cmd == "train":
        out = a.out or NETS[a.dist]
        mlp, summary = train(d=a.d, n=a.n, datasets=a.datasets, epochs=a.epochs, lr=a.lr,
                             feat_grid=a.feature_grid, log=log, dist=a.dist)
        os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
        mlp.save(out)
        log(json.dumps({"saved": out, **summary}))
    else:
        import torch
        torch.zeros(1, device="cuda")  # bring up torch's device context before the library's calls
        mlp = sky.MLP.load(a.net or NETS[a.dist])
        evaluate(mlp, n=a.n, d=mlp.d, k=a.k, log=log, dist=a.dist)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
