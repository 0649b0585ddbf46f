"""GPU parity of symmetry breaking (Sec. 5.4) against the CPU oracle:
queries with inequality filters on every path (depth-first count and
enumerate, the batched pipeline, the server, delta queries through the fused
and the depth-first path), and the undirected and degree-ordered graph builds
bit-exact against the oracle's transform."""
import ctypes

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


@pytest.fixture(scope="module")
def ctx(gj):
    return gj.Context(0)


def _dev(p, n):
    hip = ctypes.CDLL("libamdhip64.so")
    a = np.empty(n, np.uint32)
    if n:
        assert hip.hipMemcpy(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(p), ctypes.c_size_t(a.nbytes), 2) == 0
    return a


def fwd_edges(G):
    E = G.info()["edges"]
    rp, col, row = G.csr_ptrs(0)
    return _dev(row, E), _dev(col, E)


def rand_less(rng, m):
    pairs = [(x, y) for x in range(m) for y in range(m) if x != y]
    k = int(rng.integers(1, 4))
    return [pairs[i] for i in rng.choice(len(pairs), k, replace=False)]


def check_static(gj, ctx, G, O, q, enumerate_=True):
    ref = oracle.run(O, q, collect=enumerate_, threads=8)
    Qh = gj.Query(ctx, *q)
    c = gj.count(ctx, G, Qh)
    assert (c["matches"], c["prefixes"], c["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"]), q
    if enumerate_:
        st, rows = gj.enumerate_rows(ctx, G, Qh)
        assert np.array_equal(np.asarray(rows), ref["rows"]), q
    return ref


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4",
                                  "house", "reciprocal"])
def test_inequalities_static(gj, ctx, name):
    """Random inequality sets and orders on an R-MAT graph (several tiles of
    prefixes, skewed rows), and the symmetry-breaking sets on its undirected
    form: counts, per-stage counters and sorted rows equal the oracle's."""
    rng = np.random.default_rng(len(name))
    src, dst = synth.rmat_draws(10, seed=3)
    n = 1 << 10
    q = Q.ALL[name]
    G, O = gj.Graph(ctx, src, dst, n), oracle.Graph(n, src, dst)
    orders = Q.valid_orders(q)
    for order in [orders[0], orders[len(orders) // 2], orders[-1]]:
        check_static(gj, ctx, G, O, Q.with_less(Q.with_order(q, order), rand_less(rng, q[0])),
                     enumerate_=q[0] < 5)
    if name in Q.SYM_LESS:
        u, v = oracle.symmetric_edges(n, src, dst)
        Gu, Ou = gj.Graph(ctx, src, dst, n, undirected=True), oracle.Graph(n, u, v)
        less, aut = Q.SYM_LESS[name]
        ref = check_static(gj, ctx, Gu, Ou, Q.with_less(q, less), enumerate_=False)
        assert gj.count(ctx, Gu, gj.Query(ctx, *q))["matches"] == aut * ref["matches"]


def test_inequalities_batched_and_served(gj):
    """The batched pipeline and the server count inequality queries (mixed
    with plain ones) exactly as the oracle does over each seed slice."""
    c = gj.Context(0)
    src, dst = synth.rmat_draws(11, seed=5)
    n = 1 << 11
    u, v = oracle.symmetric_edges(n, src, dst)
    G, O = gj.Graph(c, src, dst, n, undirected=True), oracle.Graph(n, u, v)
    qs = [Q.with_less(Q.ALL[k], Q.SYM_LESS[k][0]) for k in ("triangle", "clique4", "house")]
    qs += [Q.ALL["clique4"], Q.with_less(Q.ALL["diamond"], [(1, 2)])]
    hs = [gj.Query(c, *q) for q in qs]
    E = G.info()["edges"]
    rng = np.random.default_rng(8)
    reqs = []
    for i in range(40):
        k = i % len(qs)
        lo = int(rng.integers(0, E))
        reqs.append((k, lo, lo + int(rng.integers(1, 600))))
    want = [oracle.run(O, qs[k], seed_lo=lo, seed_hi=hi, threads=8)["matches"] for k, lo, hi in reqs]
    counts, _ = gj.run_batch(c, G, [(hs[k], lo, hi) for k, lo, hi in reqs])
    assert counts == want
    S = gj.Server(c, G, max_batch=16)
    tickets = [S.submit_count(hs[k], lo, hi) for k, lo, hi in reqs]
    got = [S.wait(t)["count"] for t in tickets]
    S.close()
    assert got == want


@pytest.mark.parametrize("fused,rows", [(1, False), (0, True)])
def test_inequalities_delta(gj, fused, rows):
    """Delta queries with inequalities, count-only through the fused pipeline
    and with rows through the depth-first path: count deltas, counters and
    signed rows equal the oracle's; the undirected graph takes each change in
    both directions."""
    c = gj.Context(0)
    c.set_option("delta_fused", fused)
    scale = 10
    src, dst = synth.rmat_draws(scale, seed=6)
    n = 1 << scale
    u, v = oracle.symmetric_edges(n, src, dst)
    G, O = gj.Graph(c, src, dst, n, undirected=True), oracle.Graph(n, u, v)
    qs = [Q.with_less(Q.ALL[k], Q.SYM_LESS[k][0]) for k in ("triangle", "clique4", "clique5")]
    qs.append(Q.with_less(Q.ALL["cycle4"], [(0, 2), (1, 3)]))
    hs = [gj.Query(c, *q) for q in qs]
    for k, bs, bd, bg in synth.update_stream(scale, 6, 7, 4, 1, 800):
        keep = bs != bd
        bs, bd, bg = bs[keep], bd[keep], bg[keep]
        # an undirected change: both directions, conflicts dropped
        key = np.minimum(bs, bd).astype(np.int64) << 32 | np.maximum(bs, bd)
        _, first = np.unique(key, return_index=True)
        bs, bd, bg = bs[first], bd[first], bg[first]
        s2, d2, g2 = np.concatenate([bs, bd]), np.concatenate([bd, bs]), np.concatenate([bg, bg])
        res = gj.apply_updates(c, G, s2, d2, g2, hs, rows=rows)
        for q, r in zip(qs, res):
            ref = oracle.delta(O.copy(), s2, d2, g2, q)
            assert r["count_delta"] == ref["count_delta"], q
            assert r["stats"]["raw_emissions"] == ref["raw_emissions"], q
            assert r["stats"]["prefixes"] == ref["prefixes"] and r["stats"]["extensions"] == ref["extensions"]
            if rows:
                assert np.array_equal(r["rows"], ref["rows"]) and np.array_equal(r["signs"], ref["signs"]), q
        oracle.delta(O, s2, d2, g2)
    assert c.get_option("batch_fallbacks") == 0


def _check_build(gj, ctx, n, src, dst):
    for undirected, degree_order in ((True, False), (False, True), (True, True)):
        G = gj.Graph(ctx, src, dst, n, undirected=undirected, degree_order=degree_order)
        if degree_order:
            eu, ev, old = oracle.relabel_by_degree(n, src, dst, undirected=undirected)
        else:
            eu, ev = oracle.symmetric_edges(n, src, dst)
            old = np.arange(n, dtype=np.uint32)
        gu, gv = fwd_edges(G)
        assert np.array_equal(gu, eu) and np.array_equal(gv, ev), (n, undirected, degree_order)
        assert np.array_equal(G.vertex_ids(), old)
        info = G.info()
        deg = np.bincount(eu.astype(np.int64), minlength=n)
        ind = np.bincount(ev.astype(np.int64), minlength=n)
        assert (info["max_out"], info["max_in"]) == (int(deg.max(initial=0)), int(ind.max(initial=0)))
        G.close()


def test_builds_edge_cases(gj, ctx):
    """Empty, loops only, repeats and reciprocal pairs, one vertex, isolated
    vertices, ragged sizes over several sort tiles."""
    rng = np.random.default_rng(2)
    cases = [([], [], 5), ([1, 2, 3], [1, 2, 3], 4), ([0], [1], 2), ([0], [0], 1),
             ([0, 0, 1, 1, 2, 2, 2], [1, 1, 0, 2, 1, 0, 0], 9)]
    for n, m in ((3000, 1), (3000, 5000), (20000, 70001)):
        cases.append((rng.integers(0, n, m), rng.integers(0, n, m), n))
    for s, d, n in cases:
        _check_build(gj, ctx, n, np.asarray(s, np.uint32), np.asarray(d, np.uint32))
    plain = gj.Graph(ctx, np.array([2, 0], np.uint32), np.array([0, 1], np.uint32), 3)
    assert plain.vertex_ids().tolist() == [0, 1, 2]


def test_oriented_clique_counts(gj, ctx):
    """On the degree-ordered graph the plain clique queries (the triangle
    through the owner-grouped kernel) count each undirected clique once: the
    oracle's count on its own transform, and the undirected graph's count
    over |Aut|, with and without the inequalities."""
    src, dst = synth.rmat_draws(12, seed=9)
    n = 1 << 12
    eu, ev, _ = oracle.relabel_by_degree(n, src, dst)
    Gd, Od = gj.Graph(ctx, src, dst, n, degree_order=True), oracle.Graph(n, eu, ev)
    Gu = gj.Graph(ctx, src, dst, n, undirected=True)
    for name in ("triangle", "clique4", "clique5"):
        q = Q.ALL[name]
        less, aut = Q.SYM_LESS[name]
        ref = check_static(gj, ctx, Gd, Od, q, enumerate_=name == "triangle")
        assert ref["matches"] > 0
        assert gj.count(ctx, Gu, gj.Query(ctx, *Q.with_less(q, less)))["matches"] == ref["matches"]
        assert gj.count(ctx, Gu, gj.Query(ctx, *q))["matches"] == aut * ref["matches"]


def test_register_errors(gj, ctx):
    for less in ([(0, 0)], [(0, 3)], [(0, 1)] * 29):
        with pytest.raises(gj.GJError):
            gj.Query(ctx, *Q.with_less(Q.TRIANGLE, less))
    with pytest.raises(gj.GJError):
        gj.Graph(ctx, np.array([0], np.uint32), np.array([5], np.uint32), 3, degree_order=True)
