"""Autotuner for the grid resolution (cells per dimension) of the skyline path.

For every (d, n) on a grid of shapes it times the single-instance path on the
three synthetic distributions for each candidate grid, refine form and (for the
wave form) number of waves per work item, and keeps, per (d, n), the choice
with the lowest mean time, and for each input class (independent, correlated,
anti-correlated: the library computes a call's class from a sample of its
input, skycell_input_class) the choice fastest on that class.  The result is
a text table of
"d log2n dtype g form parts [class]" lines that the library loads with
skycell_load_tuning (form: the refine form, 0 lane, 1 wave; parts: waves per
item of the wave form; class: for single calls, one more row per input class
whose own fastest configuration differs from the one with the lowest mean):

    dtype 0 = binary32, single-instance calls (skycell_compute with grid_res 0)
    dtype 2 = binary32, instances of a batched plan

dtype 2 rows come from a second sweep that times batched plans of 24
instances of each shape (throughput under sharing, not one call's latency).

Run on the GPU the table is meant for:

    python -m paper_2107_09993_amd.autotune --out paper_2107_09993_amd/tuning/mi355x.txt
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_TABLE = os.path.join(HERE, "tuning", "mi355x.txt")


def candidate_grids(n, d, max_cells):
    out = []
    for g in (1, 2, 3, 4, 5, 6, 8, 10, 12, 16, 24, 32, 48, 64):
        r = (g - 1).bit_length()
        if (1 << (r * d)) <= max_cells:
            out.append(g)
    return out


def time_once(sky, torch, soa, n, d, g, reps):
    s = sky.Skyline(n, d, grid_res=g, device=soa.device)
    s.run(soa)
    s.result()
    best = math.inf
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.run(soa)
        s.result()
        best = min(best, time.perf_counter() - t0)
    return best


def time_batched(sky, torch, arrays, g, reps):
    """Seconds per instance of one graph launch over `arrays` (all with grid g):
    the instances of a batched plan share the chip, so what counts there is
    throughput, not one instance's latency."""
    dev = torch.device("cuda:0")
    plan = sky.BatchedPlan([a.shape[0] for a in arrays], [a.shape[1] for a in arrays],
                           grid_res=[g] * len(arrays), device=dev)
    buf = plan.pack(arrays)
    plan.run(buf)  # captures the graph
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        t0 = time.perf_counter()
        plan.run(buf)
        torch.cuda.synchronize()
        best = min(best, time.perf_counter() - t0)
    plan.close()
    return best / len(arrays)


FORMS = ("lane", "wave")
WAVE_PARTS = (1, 2, 4, 8, 16)
BATCH_SEEDS = 8  # instances per distribution in a batched timing


def sweep_batched(dims, sizes, reps=2, log=print):
    """Per (d, n): the configuration with the highest throughput when
    3 * BATCH_SEEDS instances of that shape run as one batched plan."""
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    table = []
    for d in dims:
        for n in sizes:
            max_cells = min(1 << 24, max(1 << 16, 32 * n))
            grids = candidate_grids(n, d, max_cells)
            configs = [(g, "lane", 1) for g in grids] + [(g, "wave", p) for g in grids for p in WAVE_PARTS]
            arrays = [datagen.generate(dist, n, d, seed=200 + 10 * k + j)
                      for k, dist in enumerate(datagen.DISTRIBUTIONS) for j in range(BATCH_SEEDS)]
            per = {}
            for g, f, p in configs:
                sky.set_refine_form(f)
                sky.set_wave_parts(p)
                per[(g, f, p)] = time_batched(sky, torch, arrays, g, reps)
            sky.set_refine_form("auto")
            sky.set_wave_parts(0)
            best = min(configs, key=lambda c: per[c])
            l2 = int(round(math.log2(n)))
            table.append((d, l2, best[0], FORMS.index(best[1]), best[2]))
            log(json.dumps({"batched": True, "d": d, "n": n, "best": "%d/%s/%d" % best,
                            "ms_per_instance": {"%d/%s/%d" % c: round(1e3 * t, 4) for c, t in per.items()}}))
    return table


def sweep(dims, sizes, reps=2, log=print):
    import numpy as np
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    dev = torch.device("cuda:0")
    table = []
    for d in dims:
        for n in sizes:
            # batched instances may use up to 32 cells per point (at most 2^24);
            # single calls up to the library's 2^24-cell default budget
            max_cells = min(1 << 24, max(1 << 16, 32 * n))
            grids = candidate_grids(n, d, max_cells)
            configs = [(g, "lane", 1) for g in grids] + [(g, "wave", p) for g in grids for p in WAVE_PARTS]
            per = {dist: dict.fromkeys(configs, 0.0) for dist in datagen.DISTRIBUTIONS}
            for k, dist in enumerate(datagen.DISTRIBUTIONS):
                x = datagen.generate(dist, n, d, seed=100 + k)
                soa = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
                for g, f, p in configs:
                    sky.set_refine_form(f)
                    sky.set_wave_parts(p)
                    per[dist][(g, f, p)] = time_once(sky, torch, soa, n, d, g, reps)
                del soa
            sky.set_refine_form("auto")
            sky.set_wave_parts(0)
            totals = {c: sum(per[dist][c] for dist in datagen.DISTRIBUTIONS) for c in configs}
            best = min(configs, key=lambda c: totals[c])
            l2 = int(round(math.log2(n)))
            table.append((d, l2, best[0], FORMS.index(best[1]), best[2]))
            # one more row per input class whose own best differs from the row
            # for all classes (the class index is datagen.DISTRIBUTIONS' order)
            for cls, dist in enumerate(datagen.DISTRIBUTIONS):
                own = min(configs, key=lambda c: per[dist][c])
                if own != best:
                    table.append((d, l2, own[0], FORMS.index(own[1]), own[2], cls))
            log(json.dumps({"d": d, "n": n, "best": "%d/%s/%d" % best,
                            "mean_ms": {"%d/%s/%d" % c: round(1e3 * t / 3, 3) for c, t in totals.items()},
                            "per_class_best": {dist: "%d/%s/%d" % min(configs, key=lambda c: per[dist][c])
                                               for dist in datagen.DISTRIBUTIONS}}))
    return table


def write_table(table, path, batched=None):
    """dtype 0 rows from the single-call sweep; dtype 2 rows from the batched
    sweep when given, else the single-call choices (without class rows)."""
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        f.write("# d log2n dtype g form parts [class]  -- grid resolution, refine form (0 lane, 1 wave) and\n")
        f.write("# waves per item of the wave form: dtype 0 with the lowest mean time of one call over\n")
        f.write("# the independent, correlated and anti-correlated inputs (with a class column: the\n")
        f.write("# lowest time on that input class, 0 independent, 1 correlated, 2 anti-correlated),\n")
        f.write("# dtype 2 with the highest throughput of batched plans of such instances\n")
        f.write("# (paper_2107_09993_amd.autotune)\n")
        for row in table:
            f.write("%d %d 0 %d %d %d" % (row[0], row[1], row[2], row[3], row[4]))
            f.write(" %d\n" % row[5] if len(row) > 5 else "\n")
        for row in (batched if batched is not None else [r for r in table if len(r) == 5]):
            f.write("%d %d 2 %d %d %d\n" % tuple(row[:5]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=DEFAULT_TABLE)
    ap.add_argument("--dims", default="2,3,4,5,6,7,8,9,10,11,12")
    ap.add_argument("--sizes", default="1000,4000,16000,64000,200000")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--no-batched", action="store_true", help="dtype 2 rows copy the single-call choices")
    a = ap.parse_args()
    dims = [int(v) for v in a.dims.split(",")]
    sizes = [int(v) for v in a.sizes.split(",")]
    log = lambda s: print(s, flush=True)
    table = sweep(dims, sizes, a.reps, log=log)
    batched = None if a.no_batched else sweep_batched(dims, sizes, a.reps, log=log)
    write_table(table, a.out, batched)
    print("wrote", a.out, flush=True)


if __name__ == "__main__":
    sys.path.insert(0, os.path.dirname(HERE))
    main()
