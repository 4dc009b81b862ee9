"""Write tests/golden/skylines.json: the oracle's skyline of every large
workload, stored as its size and the SHA-256 of its bytes.

Every value here comes from the CPU oracle (``oracle.skyline_kdtree``, the
orthant-emptiness test O3 on a k-d tree, checked against brute force and the
sort-first skyline by tests/test_oracle.py) run on the seeded synthetic inputs
of ``paper_2107_09993_amd.datagen``.  Nothing is taken from the GPU library.

An entry holds the input's recipe, the SHA-256 of the input array (row-major
[n, d] bytes, so a test can tell a generator difference from a skyline
difference), the skyline size and the SHA-256 of the ascending int32
(little-endian) skyline indices.  Equal hashes mean byte-equal results.

    python tests/golden/make_goldens.py            # all workloads
    python tests/golden/make_goldens.py --only H   # one entry
"""
import argparse
import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from paper_2107_09993_amd import datagen  # noqa: E402

OUT = os.path.join(HERE, "skylines.json")

# name -> (distribution, n, d, seed, quantised to u16 with 10 bits)
SINGLE = {
    "C1": ("independent", 10_000, 4, 0, False),
    "C2-ind": ("independent", 1_000_000, 8, 0, False),
    "C2-corr": ("correlated", 1_000_000, 8, 0, False),
    "C2-anti": ("anticorrelated", 1_000_000, 8, 0, False),
    "H": ("anticorrelated", 10_000_000, 8, 0, False),
    "C3": ("anticorrelated", 10_000_000, 6, 0, True),
    "C5-eval": ("anticorrelated", 20_000_000, 10, 0, False),
}


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def make_input(dist, n, d, seed, quantised):
    x = datagen.generate(dist, n, d, seed)
    return datagen.quantise_u16(x) if quantised else x


def entry(x, recipe):
    t0 = time.time()
    idx = oracle.skyline_kdtree(x)
    return dict(recipe, input_sha256=sha(x), count=int(idx.size),
                skyline_sha256=sha(idx.astype("<i4")), oracle="O3 k-d tree orthant test",
                oracle_seconds=round(time.time() - t0, 2))


def batched_entries(count=4096):
    out = []
    for b, (n, d, dist, seed) in enumerate(datagen.batched_instances(count=count)):
        x = datagen.generate(dist, n, d, seed)
        idx = oracle.skyline_kdtree(x)
        out.append([int(idx.size), sha(idx.astype("<i4")), sha(x)])
        if b % 256 == 255:
            print("batched %d/%d" % (b + 1, count), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="", help="comma-separated entry names (C4 = the batched workload)")
    a = ap.parse_args()
    want = set(filter(None, a.only.split(",")))
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    data.setdefault("single", {})
    for name, (dist, n, d, seed, q) in SINGLE.items():
        if want and name not in want:
            continue
        x = make_input(dist, n, d, seed, q)
        recipe = {"dist": dist, "n": n, "d": d, "seed": seed, "dtype": "u16" if q else "f32",
                  "value_bits": 10 if q else None}
        data["single"][name] = entry(x, recipe)
        print(name, data["single"][name]["count"], data["single"][name]["oracle_seconds"], "s", flush=True)
        del x
    if not want or "C4" in want:
        t0 = time.time()
        data["C4"] = {"recipe": "datagen.batched_instances(count=4096): per instance [count, skyline sha256, "
                                "input sha256]", "instances": batched_entries()}
        print("C4", round(time.time() - t0, 1), "s", flush=True)
    with open(OUT, "w") as f:
        json.dump(data, f, indent=0, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
