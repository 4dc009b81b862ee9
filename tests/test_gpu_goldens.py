"""Byte-equal parity of the HIP path with the CPU oracle at the full sizes of
every workload, against stored oracle results.

tests/golden/skylines.json holds, for each workload, the SHA-256 of its input
array and of the oracle's skyline (ascending int32 indices), written by
tests/golden/make_goldens.py from the CPU oracle alone (the k-d tree orthant
test O3, itself checked against brute force and the sort-first skyline in
tests/test_oracle.py).  Equal hashes and sizes mean byte-equal results.  On a
mismatch the test recomputes the oracle here and names the first indices that
differ.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import paper_2107_09993_amd as sky
from paper_2107_09993_amd import datagen

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "skylines.json")
GOLDEN = json.load(open(GOLDEN_PATH)) if os.path.exists(GOLDEN_PATH) else {"single": {}, "C4": {"instances": []}}


def _dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(GOLDEN_PATH):
        pytest.fail("tests/golden/skylines.json is missing (tests/golden/make_goldens.py writes it)")
    return torch.device("cuda:0")


def sha(a):
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def make_input(e):
    x = datagen.generate(e["dist"], e["n"], e["d"], e["seed"])
    return datagen.quantise_u16(x) if e["dtype"] == "u16" else x


def assert_golden(x, got, e, what):
    got = np.ascontiguousarray(got, dtype="<i4")
    if got.size == e["count"] and sha(got) == e["skyline_sha256"]:
        return
    import oracle
    ref = oracle.skyline_kdtree(x)
    diff = np.setxor1d(ref, got)[:20]
    raise AssertionError("%s: GPU skyline of %d points, oracle %d; first differing indices %s"
                         % (what, got.size, ref.size, diff.tolist()))


@pytest.fixture(scope="module")
def inputs():
    """Inputs of the single-instance workloads, generated once and checked
    against the stored input hashes."""
    cache = {}

    def get(name):
        _dev()
        if name not in cache:
            e = GOLDEN["single"][name]
            x = make_input(e)
            assert sha(x) == e["input_sha256"], "%s: the generator produced other data" % name
            cache.clear()  # keep one large input alive at a time
            cache[name] = x
        return cache[name]
    return get


def run_plain(x, grid_res=0, value_bits=10):
    dev = _dev()
    n, d = x.shape
    t = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    s = sky.Skyline(n, d, dtype="f32" if x.dtype == np.float32 else "u16", grid_res=grid_res,
                    value_bits=value_bits, device=dev)
    s.run(t)
    out = s.result().cpu().numpy()
    del s, t
    torch.cuda.empty_cache()
    return out


@pytest.mark.parametrize("name", ["C1", "C2-ind", "C2-corr", "C2-anti", "H", "C3", "C5-eval"])
def test_single_workload_full(inputs, name):
    """Every single-instance workload, at its full size and in the launch
    configuration the benchmark uses (grid chosen by the library)."""
    e = GOLDEN["single"][name]
    x = inputs(name)
    assert_golden(x, run_plain(x, grid_res=8 if name == "C1" else 0), e, name)


@pytest.mark.parametrize("name,grid", [("C2-anti", 4), ("C2-ind", 6), ("H", 6), ("C3", 8)])
def test_single_workload_other_grids(inputs, name, grid):
    e = GOLDEN["single"][name]
    x = inputs(name)
    assert_golden(x, run_plain(x, grid_res=grid), e, "%s at g = %d" % (name, grid))


@pytest.mark.parametrize("name,cls", [("C2-ind", 0), ("C2-corr", 1), ("C2-anti", 2)])
def test_c2_class_tuned_configurations(inputs, name, cls):
    """The library classifies each C2 input, and the configuration tuned for
    that class (through the Python binding, and through skycell_compute with
    grid_res = 0, which classifies the input itself) gives the oracle's
    skyline."""
    import ctypes
    e = GOLDEN["single"][name]
    x = inputs(name)
    dev = _dev()
    n, d = x.shape
    soa = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    assert sky.input_class(soa) == cls
    g, form, parts = sky.choose_config(n, d, sky.DTYPE_F32, cls)
    sky.set_refine_form(form)
    sky.set_wave_parts(parts if form == "wave" else 0)
    try:
        got = run_plain(x, grid_res=g)
    finally:
        sky.set_refine_form("auto")
        sky.set_wave_parts(0)
    assert_golden(x, got, e, "%s with its class configuration g = %d, %s" % (name, g, form))
    idx = torch.empty(n, dtype=torch.int32, device=dev)
    cnt = torch.empty(1, dtype=torch.int32, device=dev)
    st = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rc = sky.lib().skycell_compute(ctypes.c_void_p(soa.data_ptr()), n, d, 0, ctypes.c_void_p(idx.data_ptr()),
                                   ctypes.c_void_p(cnt.data_ptr()), st)
    assert rc == sky.OK
    c = int(cnt.item())
    assert_golden(x, idx[:c].cpu().numpy(), e, "%s through skycell_compute" % name)


@pytest.mark.parametrize("form", ["lane", "wave"])
def test_c2_anti_both_refine_forms(inputs, form):
    e = GOLDEN["single"]["C2-anti"]
    x = inputs("C2-anti")
    sky.set_refine_form(form)
    try:
        got = run_plain(x, grid_res=4)
    finally:
        sky.set_refine_form("auto")
    assert_golden(x, got, e, "C2-anti, %s refine" % form)


def test_c5_eval_pivoted_by_the_shipped_network(inputs):
    """The learned workload: 2e7 x 10 anti-correlated with the network trained on
    anti-correlated data, k = 4096 pivots; gated (default) and with the full
    pre-filter pass forced, both byte-equal to the oracle."""
    from paper_2107_09993_amd import learned
    dev = _dev()
    e = GOLDEN["single"]["C5-eval"]
    x = inputs("C5-eval")
    xs = torch.from_numpy(np.ascontiguousarray(x.T)).to(dev)
    net = sky.MLP.load(learned.NETS["anticorrelated"])
    got, st = sky.compute_pivoted(xs, net, k=4096, return_stats=True)
    assert_golden(x, got.cpu().numpy(), e, "C5-eval pivoted (gated)")
    sky.set_pivot_gate(False)
    try:
        got, st2 = sky.compute_pivoted(xs, net, k=4096, return_stats=True)
    finally:
        sky.set_pivot_gate(True)
    assert_golden(x, got.cpu().numpy(), e, "C5-eval pivoted (full pre-filter)")
    assert st2["skyline"] == e["count"]
    assert st2["pivot_removed"] <= e["n"] - e["count"]  # only non-skyline points can go
    net.close()


def test_c4_all_4096_instances():
    """The batched workload: all 4,096 instances in one graph launch, each
    byte-equal to the oracle."""
    dev = _dev()
    shapes = datagen.batched_instances(count=4096)
    want = GOLDEN["C4"]["instances"]
    assert len(want) == len(shapes)
    plan = sky.BatchedPlan([s[0] for s in shapes], [s[1] for s in shapes], device=dev)
    buf = np.empty(int(plan.points_off[-1]), dtype=np.float32)
    bad_inputs = []
    for b, (n, d, dist, seed) in enumerate(shapes):
        x = datagen.generate(dist, n, d, seed)
        if sha(x) != want[b][2]:
            bad_inputs.append(b)
        buf[plan.points_off[b]:plan.points_off[b + 1]] = x.T.reshape(-1)
    assert not bad_inputs, "generator produced other data for instances %s" % bad_inputs[:10]
    points = torch.from_numpy(buf).to(dev)
    del buf
    plan.run(points)
    got = plan.results()
    plan.close()
    wrong = [b for b in range(len(shapes))
             if got[b].size != want[b][0] or sha(np.ascontiguousarray(got[b], dtype="<i4")) != want[b][1]]
    assert not wrong, "instances differing from the oracle: %s" % [(b, shapes[b][:3]) for b in wrong[:10]]
