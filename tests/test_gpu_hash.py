"""Membership index (per-row hash tables, option "hash_index") against the
row searches and the oracle: counts, every counter and enumerated rows of
queries whose stages test membership, on R-MAT graphs with hub rows, over
seed slices, in the fused batch path and for delta queries reading an
indexed old version; and its invalidation when a version is rewritten."""
import numpy as np
import pytest

import oracle
import synth
from tests import queries as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gj():
    import paper_1802_03760_amd as gj
    return gj


def ctx_pair(gj):
    on, off = gj.Context(0), gj.Context(0)
    on.set_option("hash_build_work", 0)  # index at the first read that probes
    off.set_option("hash_index", 0)
    on.set_option("strategy", 1)  # the generic kernels, where the index is probed
    off.set_option("strategy", 1)
    return on, off


def stage_bindings(q):
    """Atoms binding each attribute after the first two, in the order."""
    m, atoms, order = q[0], q[1], q[2]
    pos = {a: i for i, a in enumerate(order)}
    return [[at for at in atoms if max(pos[at[0]], pos[at[1]]) == j] for j in range(2, m)]


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4", "house",
                                  "reciprocal", "clique5"])
def test_counts_rows_and_counters(gj, name):
    q = Q.ALL[name]
    scale = 12
    src, dst = synth.rmat_draws(scale, seed=31)
    n = 1 << scale
    O = oracle.Graph(n, src, dst)
    E = O.num_edges
    on, off = ctx_pair(gj)
    Gon, Goff = gj.Graph(on, src, dst, n), gj.Graph(off, src, dst, n)
    qon, qoff = gj.Query(on, *q), gj.Query(off, *q)
    width = 3000 if q[0] <= 3 else 200
    for lo, hi in ((0, width), (E // 3, E // 3 + width), (E - width, E)):
        ref = oracle.run(O, q, collect=True, seed_lo=lo, seed_hi=hi, threads=8)
        a = gj.count(on, Gon, qon, lo, hi)
        b = gj.count(off, Goff, qoff, lo, hi)
        for r in (a, b):
            assert (r["matches"], r["prefixes"], r["extensions"]) == (ref["matches"], ref["prefixes"],
                                                                      ref["extensions"]), (name, lo)
        st, rows = gj.enumerate_rows(on, Gon, qon, lo, hi)
        assert np.array_equal(rows, ref["rows"]), (name, lo)
    assert on.get_option("hash_builds") == (1 if any(len(b) > 1 for b in stage_bindings(q)) else 0)
    assert off.get_option("hash_builds") == 0
    for c, G in ((on, Gon), (off, Goff)):
        G.close()
        c.close()


def test_hub_rows_and_batch(gj):
    """A 20,000-entry hub row in both directions plus R-MAT background:
    the tables of hub rows span many buckets; fused batches of mixed
    queries equal the oracle."""
    rng = np.random.default_rng(4)
    n = 30000
    hub = np.zeros(20000, np.uint32)
    leaves = rng.choice(np.arange(1, n, dtype=np.uint32), 20000, replace=False)
    bs, bd = synth.rmat_draws(13, seed=8)
    src = np.concatenate([hub, leaves, bs % n, rng.integers(1, n, 60000).astype(np.uint32)])
    dst = np.concatenate([leaves, hub, bd % n, rng.integers(1, n, 60000).astype(np.uint32)])
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("hash_build_work", 0)
    G = gj.Graph(c, src, dst, n)
    qs = {k: gj.Query(c, *Q.ALL[k]) for k in ("clique4", "diamond", "cycle4", "triangle")}
    reqs = [(qs["clique4"], 0, 400), (qs["diamond"], 0, 50), (qs["cycle4"], 100, 160),
            (qs["triangle"], 0, 20000), (qs["clique4"], 20000, 30000)]
    counts, stats = gj.run_batch(c, G, reqs)
    for (h, lo, hi), k, got, st in zip(reqs, ("clique4", "diamond", "cycle4", "triangle", "clique4"), counts, stats):
        ref = oracle.run(O, Q.ALL[k], seed_lo=lo, seed_hi=hi, threads=8)
        assert got == ref["matches"] and st["extensions"] == ref["extensions"], (k, lo)
        r = gj.count(c, G, h, lo, hi)
        assert r["matches"] == ref["matches"] and r["prefixes"] == ref["prefixes"], (k, lo)
    G.close()
    c.close()


def test_delta_reads_indexed_old_version_and_invalidation(gj):
    """A count builds the index of the base version; an update's delta
    queries read it for the old version; the rewritten slot's stale index is
    never used: counts after each batch equal the oracle's."""
    scale = 11
    n = 1 << scale
    src, dst = synth.rmat_draws(scale, seed=12)
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("strategy", 1)
    c.set_option("hash_build_work", 0)
    G = gj.Graph(c, src, dst, n)
    k4 = gj.Query(c, *Q.CLIQUE4)
    for k, bs, bd, bg in synth.update_stream(scale, 12, 3, 8, 10, 3000):
        assert gj.count(c, G, k4)["matches"] == oracle.run(O, Q.CLIQUE4, threads=8)["matches"], k
        ref = oracle.delta(O, bs, bd, bg, Q.CLIQUE4)
        got = gj.apply_updates(c, G, bs, bd, bg, [k4], rows=True)[0]
        assert got["count_delta"] == ref["count_delta"], k
        assert np.array_equal(got["rows"], ref["rows"]) and np.array_equal(got["signs"], ref["signs"]), k
    assert gj.count(c, G, k4)["matches"] == oracle.run(O, Q.CLIQUE4, threads=8)["matches"]
    assert c.get_option("hash_builds") == 9  # one per version counted
    G.close()
    c.close()


def test_adaptive_build(gj):
    """With the default policy a version's index is built only once its
    static reads have proposed hash_build_work candidates per edge: small
    slices build none, repeated whole counts build one, an update makes the
    next version start from zero."""
    scale = 12
    n = 1 << scale
    src, dst = synth.rmat_draws(scale, seed=40)
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("strategy", 1)
    G = gj.Graph(c, src, dst, n)
    E = G.info(degrees=False)["edges"]
    k4 = gj.Query(c, *Q.CLIQUE4)
    ref = oracle.run(O, Q.CLIQUE4, threads=8)
    assert gj.count(c, G, k4, 0, 5)["matches"] == oracle.run(O, Q.CLIQUE4, seed_lo=0, seed_hi=5)["matches"]
    assert c.get_option("hash_builds") == 0
    # both stages of the 4-clique probe; the account of one whole count
    per = ref["extensions"][2] + ref["extensions"][3]
    f = max(1, (7 * per) // (2 * E))  # about 3.5 whole counts' worth per edge
    c.set_option("hash_build_work", f)
    need = -(-f * E // per)
    assert f * E > per and need >= 2
    for i in range(need + 1):
        r = gj.count(c, G, k4)
        assert (r["matches"], r["extensions"]) == (ref["matches"], ref["extensions"])
    assert c.get_option("hash_builds") == 1
    bs, bd, bg = synth.update_batch(scale, 40, 16 << scale, 2, 0, 500)
    oracle.delta(O, bs, bd, bg)
    gj.apply_updates(c, G, bs, bd, bg, [k4])
    assert gj.count(c, G, k4)["matches"] == oracle.run(O, Q.CLIQUE4, threads=8)["matches"]
    assert c.get_option("hash_builds") == 1
    G.close()
    c.close()
