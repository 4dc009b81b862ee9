"""Write tests/golden/quadrants.json: the oracle's answers to the quadrant
skyline queries of Section VII-B3 on one seeded data set.

Query q takes origin o_q and the closed top-right quadrant
Q(o_q) = { p : p[k] >= o_q[k] for every k }; its answer is the skyline of Q(o_q)
(Definitions 1-2), as ascending indices into the data set.  Every answer here
comes from the CPU oracle (``oracle.skyline_sfs`` on the points of the
quadrant, selected with numpy); nothing is taken from the GPU library.

Stored: the recipe, the SHA-256 of the data and of the origins, every query's
quadrant size and skyline size, and one SHA-256 over all answers (each as
little-endian int32 indices, in query order).  Equal hashes mean every query's
answer is byte-equal.

    python tests/golden/make_quadrant_goldens.py
"""
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2107_09993_amd import datagen  # noqa: E402

OUT = os.path.join(HERE, "quadrants.json")
RECIPE = {"dist": "independent", "n": 100_000, "d": 4, "seed": 0, "queries": 10_000, "origin_seed": 1}


def make_data(r):
    x = datagen.generate(r["dist"], r["n"], r["d"], r["seed"])
    o = np.random.default_rng(r["origin_seed"]).random((r["queries"], r["d"]), dtype=np.float32)
    return x, o


def answer(x, o):
    ids = np.nonzero((x >= o).all(axis=1))[0]
    if ids.size == 0:
        return ids.astype(np.int32), 0
    return ids[oracle.skyline_sfs(x[ids], nthreads=1)].astype(np.int32), int(ids.size)


def answers(x, origins, threads=None):
    threads = threads or oracle.default_threads()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(lambda q: answer(x, origins[q]), range(origins.shape[0])))


def digest(skylines):
    h = hashlib.sha256()
    for s in skylines:
        h.update(np.ascontiguousarray(s, dtype="<i4").tobytes())
        h.update(b"|")
    return h.hexdigest()


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main():
    x, o = make_data(RECIPE)
    t0 = time.time()
    res = answers(x, o)
    out = dict(RECIPE, data_sha256=sha(x), origins_sha256=sha(o),
               quadrant_sizes=[r[1] for r in res], skyline_sizes=[int(r[0].size) for r in res],
               answers_sha256=digest([r[0] for r in res]), oracle="sort-first skyline (O2) per quadrant",
               oracle_seconds=round(time.time() - t0, 1))
    with open(OUT, "w") as f:
        json.dump(out, f)
    print("wrote %s (%d queries, %.1f s)" % (OUT, len(res), time.time() - t0))


if __name__ == "__main__":
    main()
