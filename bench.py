#!/usr/bin/env python3
"""Benchmark of the exact-skyline path on one MI355X.

A step is one complete skyline call (quantise + histogram, cell prune, scan,
scatter, refine, ordered output) over the resident input, followed by reading
the skyline size back.  The workload is n = 10^7 anti-correlated points in d = 8
(seeded synthetic data, generated on the host and copied to HBM before timing).

Prints one JSON line.  `value` is input points per second over the K timed
steps (wall clock between two device synchronisations).  `roofline` describes
the dominant kernel (the refine), timed with hipEvents recorded on the launch
stream during the timed steps; `cpu_baseline` is the CPU oracle (its k-d tree
orthant test) timed on the same data.  `configs` times the other
single-instance workloads the same way (points/s, dominance tests/s, bandwidth
of the algorithmic bytes); `batched` and `learned` are the batched and
learned-proposer workloads.  Progress lines go to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "input points/sec to exact skyline (n=10M, d=8 anti-corr); batched instances/sec"

# MI355X: 256 compute units at 2.4 GHz, 64 lanes per CU per clock for 32-bit
# integer compare/ALU instructions (no packing).
PEAK_ALU_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12


def progress(msg):
    """One line per finished leg on stderr, so a long run shows where it is."""
    print("[bench %.1fs] %s" % (time.perf_counter() - T_START, msg), file=sys.stderr, flush=True)


T_START = time.perf_counter()


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=10_000_000)
    ap.add_argument("--d", type=int, default=8)
    ap.add_argument("--dist", default="anticorrelated")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--cpu-sample", type=int, default=-1,
                    help="points of the workload for the CPU oracle baseline (-1 = all of "
                         "them, 0 = skip)")
    ap.add_argument("--configs", type=int, default=1,
                    help="also time the other single-instance workloads (1 = yes)")
    ap.add_argument("--config-steps", type=int, default=10)
    ap.add_argument("--batched-count", type=int, default=4096,
                    help="instances of the batched workload (0 = skip)")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--learned-n", type=int, default=20_000_000,
                    help="points of the learned-proposer evaluation (0 = skip)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run three device-to-device copies of 1 GiB (the reference "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("refine.hip", "refine_core.h", "refine_mc.h", "common.h"):
        with open(os.path.join(ROOT, "paper_2107_09993_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            t = json.load(f)
        e = t.get(kernel, {}).get(workload)
        if e and e.get("source_hash") == kernel_source_hash():
            return e.get("bytes_per_launch")
    except (ValueError, OSError):
        return None
    return None


def batched_bench(count, steps, dev):
    """Batched workload: `count` instances with n log-uniform in [1,000, 200,000],
    d uniform in 3..12 and the distribution drawn per instance, run as one graph
    launch per step."""
    import numpy as np
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    shapes = datagen.batched_instances(count=count)
    ns = [s[0] for s in shapes]
    ds = [s[1] for s in shapes]
    plan = sky.BatchedPlan(ns, ds, device=dev)
    buf = np.empty(int(plan.points_off[-1]), dtype=np.float32)
    for b, (n, d, dist, seed) in enumerate(shapes):
        buf[plan.points_off[b]:plan.points_off[b + 1]] = datagen.generate(dist, n, d, seed).T.reshape(-1)
    points = torch.from_numpy(buf).to(dev)
    del buf
    t0 = time.perf_counter()
    plan.run(points)  # first run: captures the graph
    torch.cuda.synchronize()
    capture_s = time.perf_counter() - t0
    total_sky = int(plan.out_count.to(torch.int64).sum().item())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.run(points)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.close()
    return {"value": count * steps / wall, "unit": "instances/s", "instances": count,
            "points": int(sum(ns)), "skyline_points": total_sky, "steps": steps,
            "ms_per_launch": 1e3 * wall / steps, "first_run_with_capture_s": capture_s,
            "workload": "batched: n log-uniform in [1e3, 2e5], d uniform in 3..12, "
                        "independent/correlated/anti-correlated per instance, seeds 1e6+b"}


# The other single-instance workloads: name -> (distribution, n, d, seed, uint16 with
# 10 value bits, grid or 0 for the library's choice)
CONFIGS = {
    "C1 independent n=1e4 d=4 g=8": ("independent", 10_000, 4, 0, False, 8),
    "C2 independent n=1e6 d=8": ("independent", 1_000_000, 8, 0, False, 0),
    "C2 correlated n=1e6 d=8": ("correlated", 1_000_000, 8, 0, False, 0),
    "C2 anti-correlated n=1e6 d=8": ("anticorrelated", 1_000_000, 8, 0, False, 0),
    "C3 anti-correlated uint16 n=1e7 d=6": ("anticorrelated", 10_000_000, 6, 0, True, 0),
}


def tuned_config(sky, soa, grid):
    """The configuration a grid_res = 0 call uses on this input: its input class
    from a sample on the device, then the tuning table's grid, refine form and
    waves per item for that class (chosen once per workload, as a caller with a
    persistent workspace would).  With an explicit grid: that grid and the
    library's form choice."""
    import torch
    d, n = soa.shape
    if grid:
        return {"grid": grid, "form": None, "parts": 0, "input_class": None}
    cls = sky.input_class(soa)
    dtype = sky.DTYPE_U16 if soa.dtype == torch.uint16 else sky.DTYPE_F32
    g, form, parts = sky.choose_config(n, d, dtype, cls)
    return {"grid": g, "form": form, "parts": parts, "input_class": sky.CLASS_NAMES[cls]}


def apply_config(sky, cfg):
    """Force the configuration's refine form and waves per item (None: the
    library's per-call choice)."""
    sky.set_refine_form(cfg["form"] or "auto")
    sky.set_wave_parts(cfg["parts"] if cfg["form"] == "wave" else 0)


def single_bench(x, grid, steps, warmup, dev, value_bits=10):
    """Times `steps` calls of the whole path on resident data (one host sync per
    call, as in the headline); returns points/s, tests/s and bandwidth."""
    import numpy as np
    import torch
    import paper_2107_09993_amd as sky
    n, d = x.shape
    dtype = "u16" if x.dtype == np.uint16 else "f32"
    soa = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    cfg = tuned_config(sky, soa, grid)
    apply_config(sky, cfg)
    try:
        res = _single_bench(sky, torch, soa, n, d, dtype, cfg["grid"], steps, warmup, dev, value_bits)
    finally:
        apply_config(sky, {"form": None, "parts": 0})
    res["config"] = cfg
    return res


def _single_bench(sky, torch, soa, n, d, dtype, g, steps, warmup, dev, value_bits):
    probe = sky.Skyline(n, d, dtype=dtype, grid_res=g, value_bits=value_bits, device=dev, stats=True)
    probe.run(soa)
    count = int(probe.result().numel())
    st = probe.stats_dict()
    del probe
    sk = sky.Skyline(n, d, dtype=dtype, grid_res=g, value_bits=value_bits, device=dev)
    for _ in range(warmup):
        sk.run(soa)
        sk.result()
    sky.profile_enable(True)
    phase_sum = dict.fromkeys(sky.PHASE_NAMES, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sk.run(soa)
        c = int(sk.out_count.item())
        for k, v in sky.profile_read().items():
            phase_sum[k] += v
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sky.profile_enable(False)
    if c != count:
        raise RuntimeError("skyline size changed between calls: %d vs %d" % (c, count))
    del sk, soa
    torch.cuda.empty_cache()
    ms = 1e3 * wall / steps
    phases = {k: v / steps for k, v in phase_sum.items()}
    cells = (1 << (max(1, (g - 1).bit_length()) * d)) if g > 1 else 1
    eb = 2 if dtype == "u16" else 4
    pb = phase_bytes(n, d, cells, st)
    pb["quantize_hist"] += n * d * (eb - 4)
    pb["scatter"] += n * d * (eb - 4)
    total = sum(pb.values())
    return {"points_per_s": n / (wall / steps), "ms_per_call": ms, "grid_res": g, "dtype": dtype,
            "skyline": count, "survivor_points": st["survivor_points"],
            "dominance_tests_per_s": st["pair_tests"] / (ms * 1e-3),
            "phases_ms": phases,
            "algorithmic_bytes": total,
            "hbm_gbs": total / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": total / (ms * 1e-3) / PEAK_HBM}


def configs_bench(steps, dev):
    from paper_2107_09993_amd import datagen
    out = {}
    for name, (dist, n, d, seed, u16, grid) in CONFIGS.items():
        x = datagen.generate(dist, n, d, seed)
        if u16:
            x = datagen.quantise_u16(x)
        out[name] = single_bench(x, grid, steps, 2, dev)
        progress("config %s: %.3g points/s" % (name, out[name]["points_per_s"]))
    return out


def learned_bench(n, dev):
    """Pivoted vs plain skyline with the committed networks, k = 4096 pivots,
    with random and smallest-coordinate-sum pivots for comparison: the learned
    workload (n anti-correlated points in d = 10, trained on anti-correlated
    data) and, when its network is present, n/4 independent points in d = 10."""
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import learned
    out = {}
    for dist, npts in (("anticorrelated", n), ("independent", n // 4)):
        path = learned.NETS[dist]
        if not os.path.exists(path):
            out[dist] = {"skipped": "no trained network at %s" % path}
            continue
        mlp = sky.MLP.load(path)
        res = learned.evaluate(mlp, n=npts, d=mlp.d, k=sky.MAX_PIVOTS, reps=3, device=dev, dist=dist)
        mlp.close()
        res["workload"] = "%s n=%d d=%d seed=0, top-4096 pivots of the network trained on %s data" % (
            dist, npts, res["d"], dist)
        res["speedup_vs_plain"] = res["learned"]["speedup_vs_plain"]
        out[dist] = res
    return out


def cpu_baseline(x_host, sample):
    """The CPU oracle's k-d tree orthant test (O3) on the first `sample` points
    of the workload (all of them by default), on every host thread."""
    import oracle
    n = x_host.shape[0] if sample < 0 else min(sample, x_host.shape[0])
    xs = x_host[:n]
    threads = oracle.default_threads()
    t0 = time.perf_counter()
    sky = oracle.skyline_kdtree(xs, nthreads=threads)
    dt = time.perf_counter() - t0
    what = "all %d points" % n if n == x_host.shape[0] else "the first %d points" % n
    return {"value": n / dt, "unit": "points/s", "cores": threads, "kind": "oracle",
            "sample": "k-d tree orthant oracle (O3) on %s of the same data "
                      "(%d skyline points, %.1f s)" % (what, len(sky), dt)}


def phase_bytes(n, d, cells, st):
    """Bytes each streaming phase must move at least with this data layout
    (reads + writes, every array touched once), for the per-phase bandwidth."""
    fw = 8 * ((d + 7) // 8)
    surv = st["survivor_points"]
    # walk records are built for the lane form only (its items hold at most two
    # points, the wave form's up to 63)
    walk_records = d <= 8 and 2 * st["items"] >= surv
    return {
        # zero the counts; read the coordinates, write cell and rank per point
        "quantize_hist": 4 * cells + n * (4 * d + 8),
        # counts read, records written, the lower-closure bitmap written and
        # read once, the bitmap of surviving cells written
        "cell_prune": cells * (4 + 8) + (cells // 8) * 3,
        # record and count read, first sorted position written per cell; the
        # work items written
        "cell_scan": cells * (8 + 4 + 4) + st["items"] * 8,
        # coordinates, cell, rank, record per point; keys, screening words,
        # original index of surviving points; flag of every point; then for
        # d <= 8 the walk records (read the cell records and the screening
        # words, write one word per cell)
        "scatter": n * (4 * d + 16 + 1) + surv * (4 * d + fw + 4)
                   + (cells * 16 + surv * fw if walk_records else 0),
        # flags of every point, indices of the skyline points
        "output": n + 4 * st["skyline"],
    }


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library runs each skyline on a single "
              "MI355X and has no multi-GPU path (requested --gpus %d, WORLD_SIZE %d)"
              % (a.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2107_09993_amd as sky
    from paper_2107_09993_amd import datagen

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if a.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    x = datagen.generate(a.dist, a.n, a.d, a.seed)
    soa = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    progress("headline input generated and resident: %s n=%d d=%d" % (a.dist, a.n, a.d))
    cfg = tuned_config(sky, soa, a.grid)
    g = cfg["grid"]
    apply_config(sky, cfg)

    # one call with counters for the algorithmic work figures
    probe = sky.Skyline(a.n, a.d, grid_res=g, device=dev, stats=True)
    probe.run(soa)
    sky_count = int(probe.result().numel())
    st = probe.stats_dict()
    del probe

    sk = sky.Skyline(a.n, a.d, grid_res=g, device=dev)
    for _ in range(a.warmup):
        sk.run(soa)
        sk.result()
    torch.cuda.synchronize()

    sky.profile_enable(True)
    phase_sum = dict.fromkeys(sky.PHASE_NAMES, 0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        sk.run(soa)
        c = int(sk.out_count.item())
        ph = sky.profile_read()
        for k, v in ph.items():
            phase_sum[k] += v
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sky.profile_enable(False)
    apply_config(sky, {"form": None, "parts": 0})
    if c != sky_count:
        print("skyline size changed between calls: %d vs %d" % (c, sky_count), file=sys.stderr)
        sys.exit(1)

    ms_per_step = 1e3 * wall / a.steps
    progress("headline: %d steps, %.3f ms per step" % (a.steps, 1e3 * wall / a.steps))
    phases = {k: v / a.steps for k, v in phase_sum.items()}
    value = a.n / (wall / a.steps)

    refine_ms = phases["refine"]
    ops = st["pair_tests"] * a.d  # one compare per dimension per candidate test
    achieved = ops / (refine_ms * 1e-3)
    workload = "%s n=%d d=%d seed=%d" % (a.dist, a.n, a.d, a.seed)
    # bytes the refine must move at least: keys, screening words and original
    # index of every surviving point, the cell records (and for d <= 8 the
    # walk records), the work items, flags
    cells = (1 << (max(1, (g - 1).bit_length()) * a.d)) if g > 1 else 1
    algo_bytes = (st["survivor_points"] * (4 * a.d + 8 * ((a.d + 7) // 8) + 4) + (cells + 1) * 8
                  + (cells * 8 if a.d <= 8 else 0) + st["items"] * 8 + a.n)
    pbytes = phase_bytes(a.n, a.d, cells, st)
    phase_hbm = {k: {"algorithmic_bytes": b, "gbs": b / (phases[k] * 1e-3) / 1e9,
                     "frac_of_hbm_peak": b / (phases[k] * 1e-3) / PEAK_HBM}
                 for k, b in pbytes.items() if phases.get(k, 0.0) > 0.0}
    traffic = measured_traffic("k_refine", workload)
    kname = "k_refine<%d, 2, %s>" % (a.d, "true" if a.d <= 8 else "false")
    roof = {"kernel": kname, "bound": "alu", "achieved": achieved / 1e12,
            "peak": PEAK_ALU_OPS / 1e12, "unit": "TOP/s", "frac": achieved / PEAK_ALU_OPS,
            "traffic": traffic,
            # measured bytes per launch / launch time (rocprofv3 FETCH_SIZE + WRITE_SIZE)
            "traffic_gbs": traffic / (refine_ms * 1e-3) / 1e9 if traffic else None,
            "algorithmic_bytes": algo_bytes,
            "work": "%d candidate-vs-query domination tests x %d compares per launch"
                    % (st["pair_tests"], a.d),
            "avg_launch_ms": refine_ms}

    out = {"metric": METRIC, "value": value, "unit": "points/s", "n_gpus": 1, "steps": a.steps,
           "warmup": a.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": workload, "n": a.n, "d": a.d, "distribution": a.dist,
                      "grid_res": g, "input_class": cfg["input_class"], "skyline": sky_count},
           "phases_ms": phases,
           "phases_hbm": phase_hbm,
           "dominance_tests_per_s": st["pair_tests"] / (ms_per_step * 1e-3),
           "counters": st,
           "roofline": roof}
    del sk, soa
    torch.cuda.empty_cache()
    if a.configs:
        out["configs"] = configs_bench(a.config_steps, dev)
    if a.batched_count > 0:
        torch.cuda.empty_cache()
        out["batched"] = batched_bench(a.batched_count, a.batched_steps, dev)
        progress("batched: %.1f instances/s" % out["batched"]["value"])
    if a.learned_n > 0:
        torch.cuda.empty_cache()
        out["learned"] = learned_bench(a.learned_n, dev)
        progress("learned leg done")
    if a.cpu_sample != 0:
        out["cpu_baseline"] = cpu_baseline(x, a.cpu_sample)
        progress("cpu baseline: %.3g points/s on %d threads" % (out["cpu_baseline"]["value"],
                                                                out["cpu_baseline"]["cores"]))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
