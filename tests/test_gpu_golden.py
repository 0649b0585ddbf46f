"""Whole-graph counts and every per-stage counter at full workload sizes
against stored oracle values (tests/golden/full_counts.json, written by
tests/golden/make_golden.py from the CPU oracle alone), in the launch
configuration bench.py times: the default strategy, which sends the
triangle to the owner-grouped kernel, the 4-clique to the edge-grouped
kernels, the diamond and the 4-cycle to the 2-path kernels and the 5-clique
to the mask kernels.  Then the owner kernel with tasks cut as small as its
planning allows (every unit with more than one task's work is split), and a
hub whose single owner unit exceeds the default task size."""
import json
import os

import numpy as np
import pytest

import oracle
import synth
from tests import queries as Q
from tests.golden.make_golden import ENTRIES

pytestmark = pytest.mark.gpu

_golden = {}


def golden(name):
    if not _golden:
        path = os.path.join(os.path.dirname(__file__), "golden", "full_counts.json")
        _golden.update(json.load(open(path))["entries"])
    return _golden[name]


@pytest.fixture(scope="module")
def gj():
    import paper_1802_03760_amd as gj
    return gj


_graphs = {}


def gpu_graph(gj, ctx, spec):
    """One resident graph per spec for the module (largest first evicts)."""
    key = (id(ctx), spec["scale"], spec["build"])
    if key not in _graphs:
        for k in list(_graphs):
            _graphs.pop(k).close()
        src, dst = synth.rmat_draws(spec["scale"], spec["edge_factor"], spec["seed"])
        _graphs[key] = gj.Graph(ctx, src, dst, 1 << spec["scale"], degree_order=spec["build"] == "degree_order")
    return _graphs[key]


@pytest.fixture(scope="module")
def ctx(gj):
    c = gj.Context(0)
    yield c
    for k in list(_graphs):
        _graphs.pop(k).close()
    c.close()


# sorted so that graphs of one spec are built once
NAMES = sorted(ENTRIES, key=lambda k: (ENTRIES[k][0]["scale"], ENTRIES[k][0]["build"], k))


@pytest.mark.parametrize("name", NAMES)
def test_full_count_against_oracle(gj, ctx, name):
    g = golden(name)
    G = gpu_graph(gj, ctx, g["graph"])
    assert G.info(degrees=False)["edges"] == g["edges"]
    print("golden %s: %s, scale %d" % (name, g["query"], g["graph"]["scale"]), flush=True)
    r = gj.count(ctx, G, gj.Query(ctx, *Q.ALL[g["query"]]))
    assert r["matches"] == g["matches"], name
    assert r["prefixes"] == g["prefixes"], name
    assert r["extensions"] == g["extensions"], name
    if name == "rmat22_triangle":
        # the headline count: one owner-grouped launch, some units split into tasks
        assert r["kernel_launches"] == 1
        assert ctx.get_option("owner_split_units") > 0


@pytest.mark.parametrize("name", ["rmat20_triangle", "rmat20_cyclic_triangle"])
def test_owner_smallest_tasks_against_oracle(gj, name):
    """owner_task_min = 1: every unit whose work exceeds 8x its owner's set
    is cut into partner-range tasks (the plo > 0 path of the kernel)."""
    g = golden(name)
    c = gj.Context(0)
    c.set_option("owner_task_min", 1)
    src, dst = synth.rmat_draws(20, seed=0)
    G = gj.Graph(c, src, dst, 1 << 20)
    r = gj.count(c, G, gj.Query(c, *Q.ALL[g["query"]]))
    assert (r["matches"], r["prefixes"], r["extensions"]) == (g["matches"], g["prefixes"], g["extensions"])
    assert c.get_option("owner_split_units") > 1000
    assert c.get_option("owner_tasks") > c.get_option("owner_split_units")
    G.close()
    c.close()


@pytest.mark.parametrize("task_min", [1, 64, 1 << 20])
@pytest.mark.parametrize("scale", [13, 15])
def test_owner_task_sizes_rmat(gj, task_min, scale):
    """R-MAT 13 and 15, triangle and cyclic triangle: counts and counters
    equal the oracle's for every task size."""
    src, dst = synth.rmat_draws(scale, seed=scale)
    n = 1 << scale
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("owner_task_min", task_min)
    G = gj.Graph(c, src, dst, n)
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE):
        ref = oracle.run(O, q, threads=8)
        r = gj.count(c, G, gj.Query(c, *q))
        assert (r["matches"], r["prefixes"], r["extensions"]) == (ref["matches"], ref["prefixes"],
                                                                  ref["extensions"]), (q, task_min)
        if task_min == 1:
            assert c.get_option("owner_split_units") > 0
    G.close()
    c.close()


def hub_graph():
    """Vertex 0 has 200 out-neighbours (1..200) and 150,000 in-neighbours
    (1000..150999), each with 9 more out-edges into 1..399: every seed edge
    (x0, 0) is owned by 0 (its set out(0) is the larger), and the unit of 0
    proposes 150,000 x 10 = 1.5M values, more than one default task."""
    rng = np.random.default_rng(17)
    n = 151000
    hub_out = np.arange(1, 201, dtype=np.uint32)
    parts = np.arange(1000, 151000, dtype=np.uint32)
    extra = rng.integers(1, 400, (len(parts), 9)).astype(np.uint32)
    inner_s = rng.integers(1, 400, 4000).astype(np.uint32)
    inner_d = rng.integers(1, 400, 4000).astype(np.uint32)
    src = np.concatenate([np.zeros(200, np.uint32), parts, np.repeat(parts, 9), inner_s])
    dst = np.concatenate([hub_out, np.zeros(len(parts), np.uint32), extra.ravel(), inner_d])
    return n, src, dst


def test_owner_single_unit_split_default(gj):
    n, src, dst = hub_graph()
    ref = oracle.run(oracle.Graph(n, src, dst), Q.TRIANGLE, threads=8)
    c = gj.Context(0)
    G = gj.Graph(c, src, dst, n)
    r = gj.count(c, G, gj.Query(c, *Q.TRIANGLE))
    assert (r["matches"], r["prefixes"], r["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"])
    assert r["kernel_launches"] == 1
    assert c.get_option("owner_split_units") >= 1
    assert ref["matches"] > 0
    G.close()
    c.close()


def test_owner_signed_delta_smallest_tasks(gj):
    """Triangle deltas on the owner-grouped kernel (delta_owner_min = 1)
    with owner_task_min 1: count deltas and counters equal the oracle's
    Delta-GJ batch by batch."""
    scale = 13
    n = 1 << scale
    src, dst = synth.rmat_draws(scale, seed=2)
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("delta_owner_min", 1)
    c.set_option("owner_task_min", 1)
    G = gj.Graph(c, src, dst, n)
    q = gj.Query(c, *Q.TRIANGLE)
    for k, bs, bd, bg in synth.update_stream(scale, 2, 5, 6, 100, 20000):
        ref = oracle.delta(O, bs, bd, bg, Q.TRIANGLE, rows=False, threads=8)
        got = gj.apply_updates(c, G, bs, bd, bg, [q])[0]
        st = got["stats"]
        assert got["count_delta"] == ref["count_delta"], k
        assert st["raw_emissions"] == ref["raw_emissions"], k
        assert st["prefixes"][2] == ref["prefixes"][2] and st["extensions"][2] == ref["extensions"][2], k
        assert st["prefixes"][3] == ref["prefixes"][3], k
        assert st["kernel_launches"] == 3, k  # one owner-grouped launch per dQ_i
    G.close()
    c.close()
