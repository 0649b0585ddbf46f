"""Pins of the CPU oracle against facts fixed by the paper and by mathematics:
the paper's worked example, brute force over all vertex tuples, closed forms
on structured graphs, dense matrix identities, the delta-query identity and
order independence.  CPU only."""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import brute
from tests import queries as Q

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rand_graph(n, m, seed, loops=True):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, m).astype(np.uint32)
    d = rng.integers(0, n, m).astype(np.uint32)
    if not loops:
        keep = s != d
        s, d = s[keep], d[keep]
    return s, d


# ---------------------------------------------------------------- Appendix A
def test_appendix_a_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "appendix_a.json")))
    e = np.array(g["edges"], dtype=np.uint32)
    G = oracle.Graph(g["num_vertices"], e[:, 0], e[:, 1])
    q = (g["query"]["num_attrs"], [tuple(a) for a in g["query"]["atoms"]], g["query"]["order"])
    pr = g["printed"]
    # the printed extension sets follow from the graph
    out_ne = sorted(set(e[:, 0].tolist()))
    in_ne = sorted(set(e[:, 1].tolist()))
    assert out_ne == pr["Ext1_1_projection_out_nonempty"] == pr["Ext2_2_projection_out_nonempty"]
    assert in_ne == pr["Ext3_1_projection_in_nonempty"]
    assert sorted(e[e[:, 0] == 1, 1].tolist()) == pr["Ext1_2_of_1"]
    assert sorted(e[e[:, 0] == 6, 1].tolist()) == pr["Ext2_3_of_1_6"]
    assert sorted(e[e[:, 1] == 1, 0].tolist()) == pr["Ext3_3_of_1_6"]
    P = oracle.textbook(G, q)
    assert P[0].tolist() == pr["P1"]
    assert P[1].tolist() == pr["P2"]
    assert P[2].tolist() == pr["P3"]
    # the edge-seeded form reaches the same P_3
    r = oracle.run(G, q, collect=True)
    assert r["rows"].tolist() == pr["P3"]
    assert r["matches"] == 3


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond",
                                  "paper_diamond", "cycle4", "reciprocal"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_brute_force_small(name, seed):
    q = Q.ALL[name]
    n = 24 if q[0] == 3 else 14
    s, d = rand_graph(n, n * 5, seed)
    A = brute.adjacency(n, s, d)
    want = brute.matches(A, q)
    G = oracle.Graph(n, s, d)
    for order in Q.valid_orders(q):
        r = oracle.run(G, Q.with_order(q, order), collect=True)
        assert r["matches"] == len(want)
        assert np.array_equal(r["rows"], want), order


@pytest.mark.parametrize("name", ["house", "clique5"])
def test_brute_force_five_attrs(name):
    q = Q.ALL[name]
    n = 10
    s, d = rand_graph(n, 70, 7)
    A = brute.adjacency(n, s, d)
    want = brute.matches(A, q)
    G = oracle.Graph(n, s, d)
    r = oracle.run(G, q, collect=True)
    assert np.array_equal(r["rows"], want)
    assert len(want) > 0


def test_brute_force_n50_triangle():
    n = 50
    s, d = rand_graph(n, 600, 11)
    A = brute.adjacency(n, s, d)
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE):
        want = brute.matches(A, q)
        r = oracle.run(oracle.Graph(n, s, d), q, collect=True)
        assert np.array_equal(r["rows"], want)


def test_textbook_equals_edge_seeded():
    n = 16
    s, d = rand_graph(n, 90, 3)
    G = oracle.Graph(n, s, d)
    for name in ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4"]:
        q = Q.ALL[name]
        P = oracle.textbook(G, q)
        r = oracle.run(G, q, collect=True)
        # textbook rows are in position order == attribute order here
        assert np.array_equal(P[-1][np.lexsort(P[-1].T[::-1])], r["rows"])


# ---------------------------------------------------------------- closed forms
def complete(n):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    return s[keep].astype(np.uint32), d[keep].astype(np.uint32)


def tournament(n):
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s < d
    return s[keep].astype(np.uint32), d[keep].astype(np.uint32)


@pytest.mark.parametrize("n", [2, 3, 5, 9])
def test_complete_digraph(n):
    G = oracle.Graph(n, *complete(n))
    assert oracle.run(G, Q.TRIANGLE)["matches"] == n * (n - 1) * (n - 2)
    assert oracle.run(G, Q.CYCLIC_TRIANGLE)["matches"] == n * (n - 1) * (n - 2)
    assert oracle.run(G, Q.CLIQUE4)["matches"] == n * (n - 1) * (n - 2) * (n - 3)
    assert oracle.run(G, Q.CLIQUE5)["matches"] == n * (n - 1) * (n - 2) * (n - 3) * (n - 4)
    # the house's a4 joins a1 and a2 only: any vertex but those two
    assert oracle.run(G, Q.HOUSE)["matches"] == n * (n - 1) * (n - 2) * (n - 3) * (n - 2)
    assert oracle.run(G, Q.DIAMOND)["matches"] == (n - 1) ** 4 + (n - 1)
    assert oracle.run(G, Q.CYCLE4)["matches"] == (n - 1) ** 4 + (n - 1)


@pytest.mark.parametrize("n", [3, 6, 11])
def test_transitive_tournament(n):
    G = oracle.Graph(n, *tournament(n))
    assert oracle.run(G, Q.TRIANGLE)["matches"] == math.comb(n, 3)
    assert oracle.run(G, Q.CLIQUE4)["matches"] == math.comb(n, 4)
    assert oracle.run(G, Q.CYCLIC_TRIANGLE)["matches"] == 0
    assert oracle.run(G, Q.CYCLE4)["matches"] == 0
    want = sum((n - d) * (d - 1) ** 2 for d in range(1, n))
    assert oracle.run(G, Q.DIAMOND)["matches"] == want


def test_bipartite_odd_cycles_vanish():
    rng = np.random.default_rng(5)
    L, R = 40, 35
    s = rng.integers(0, L, 900)
    d = rng.integers(L, L + R, 900)
    flip = rng.random(900) < 0.5  # arcs in both directions across the cut
    s2 = np.where(flip, d, s).astype(np.uint32)
    d2 = np.where(flip, s, d).astype(np.uint32)
    G = oracle.Graph(L + R, s2, d2)
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE, Q.CLIQUE4):
        assert oracle.run(G, q)["matches"] == 0
    # even cycles are bipartite patterns and do occur
    assert oracle.run(G, Q.CYCLE4)["matches"] > 0
    assert oracle.run(G, Q.DIAMOND)["matches"] > 0


def test_er2000_dense_identities():
    """Workload: ER digraph, n = 2,000, 20,000 distinct arcs, seed 0.
    Counts equal dense matrix forms: transitive triangle = sum(A o A^2),
    cyclic triangle = tr(A^3), two-2-path diamond = sum((A^2)^2),
    4-cycle = tr(A^4) (exact in float64 below 2^53)."""
    s, d = synth.er_edges(2000, 20000, 0)
    A = brute.adjacency(2000, s, d).astype(np.float64)
    A2 = A @ A
    G = oracle.Graph(2000, s, d)
    r = oracle.run(G, Q.TRIANGLE, collect=True)
    assert r["matches"] == int((A * A2).sum())
    assert r["prefixes"][2] == 20000
    # the stage-3 extension counter: sum over arcs of min(out(a1), out(a2))
    outd = np.bincount(s, minlength=2000)
    assert r["extensions"][2] == int(np.minimum(outd[s], outd[d]).sum())
    # every row is a triangle
    rows = r["rows"].astype(np.int64)
    assert A[rows[:, 0], rows[:, 1]].all() and A[rows[:, 1], rows[:, 2]].all()
    assert A[rows[:, 0], rows[:, 2]].all()
    assert oracle.run(G, Q.CYCLIC_TRIANGLE)["matches"] == int(np.trace(A2 @ A))
    assert oracle.run(G, Q.DIAMOND)["matches"] == int((A2 * A2).sum())
    assert oracle.run(G, Q.CYCLE4)["matches"] == int(np.trace(A2 @ A2))


def test_agm_bound_triangle():
    s, d = synth.rmat_draws(10, seed=3)
    G = oracle.Graph(1 << 10, s, d)
    E = G.num_edges
    r = oracle.run(G, Q.TRIANGLE)
    assert r["matches"] <= E ** 1.5
    assert r["prefixes"][3] == r["matches"]


def test_gj_work_bound_triangle():
    """Generic Join's work on the triangle (Sec. 2.2): the count-minimised
    proposals of stage 2 are the sum over seed edges of min(|out(a0)|,
    |out(a1)|), at most the sum of the smaller undirected degree, which
    Chiba and Nishizeki bound by 2 a(G) |E| with arboricity a(G) <=
    ceil(sqrt(2|E| + n) / 2), so O(|E|^{3/2}).  Checked on a skewed R-MAT
    graph, a hub with reciprocal arcs to 5,000 leaves that form a path, and
    a complete digraph; on the hub graph the sum of the larger sets would
    exceed the bound more than tenfold."""
    graphs = []
    s, d = synth.rmat_draws(12, seed=8)
    graphs.append((1 << 12, s, d))
    leaves = np.arange(1, 5001, dtype=np.uint32)
    graphs.append((5001, np.concatenate([np.zeros(5000, np.uint32), leaves, leaves[:-1]]),
                   np.concatenate([leaves, np.zeros(5000, np.uint32), leaves[1:]])))
    k = 60
    a, b = np.meshgrid(np.arange(k, dtype=np.uint32), np.arange(k, dtype=np.uint32))
    graphs.append((k, a[a != b], b[a != b]))
    for n, src, dst in graphs:
        G = oracle.Graph(n, src, dst)
        E = G.num_edges
        r = oracle.run(G, Q.TRIANGLE, threads=4)
        arb = int(np.ceil(np.sqrt(2 * E + n) / 2))
        assert r["extensions"][2] <= 2 * arb * E, (n, E, r["extensions"][2])
        assert r["extensions"][2] <= 2 * E ** 1.5 + 2 * E
        # and the count-minimised sum is what it says: min, not max or sum
        u = np.unique(np.stack([src, dst], 1)[src != dst], axis=0)
        out = np.bincount(u[:, 0], minlength=n)
        assert r["extensions"][2] == int(np.minimum(out[u[:, 0]], out[u[:, 1]]).sum())
        if n == 5001:
            assert int(np.maximum(out[u[:, 0]], out[u[:, 1]]).sum()) > 10 * 2 * arb * E


# ---------------------------------------------------------------- orders, threads, slices
def test_order_and_thread_independence():
    s, d = synth.rmat_draws(9, seed=4)
    G = oracle.Graph(1 << 9, s, d)
    for q in (Q.TRIANGLE, Q.CLIQUE4, Q.CYCLE4):
        base = oracle.run(G, q, collect=True)
        for order in Q.valid_orders(q)[:6]:
            r = oracle.run(G, Q.with_order(q, order), collect=True, threads=3)
            assert np.array_equal(r["rows"], base["rows"])


def test_seed_slices_partition():
    s, d = synth.rmat_draws(9, seed=5)
    G = oracle.Graph(1 << 9, s, d)
    E = G.num_edges
    full = oracle.run(G, Q.TRIANGLE, collect=True)
    cuts = [0, 17, 400, E // 2, E]
    parts = [oracle.run(G, Q.TRIANGLE, collect=True, seed_lo=a, seed_hi=b)
             for a, b in zip(cuts[:-1], cuts[1:])]
    assert sum(p["matches"] for p in parts) == full["matches"]
    assert sum(p["extensions"][2] for p in parts) == full["extensions"][2]
    rows = np.concatenate([p["rows"] for p in parts])
    assert np.array_equal(rows[np.lexsort(rows.T[::-1])], full["rows"])


def test_invalid_queries():
    assert not oracle.query_valid((3, [(0, 1), (1, 2)], [0, 2, 1]))  # a1,a3 share no atom
    assert not oracle.query_valid((3, [(0, 0), (0, 1), (1, 2)], [0, 1, 2]))  # self-loop atom
    assert not oracle.query_valid((4, [(0, 1), (2, 3)], [0, 1, 2, 3]))  # cartesian product
    assert not oracle.query_valid((3, [(0, 1), (1, 2)], [0, 1, 1]))  # not a permutation
    assert oracle.query_valid(Q.CYCLE4)


# ---------------------------------------------------------------- delta queries
def test_delta_forced_cancellation():
    """Insert 1->2 and delete 2->3 with 1->3 present: dQ_1 emits (1,2,3) +1,
    dQ_2 emits it -1; the consolidated change is empty."""
    G = oracle.Graph(4, [2, 1], [3, 3])
    r = oracle.delta(G, [1, 2], [2, 3], [1, -1], Q.TRIANGLE)
    assert r["raw_emissions"] == 2
    assert r["count_delta"] == 0
    assert len(r["rows"]) == 0
    assert sorted(zip(*G.edge_list())) == [(1, 2), (1, 3)]


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond",
                                  "cycle4", "reciprocal"])
def test_delta_equals_recompute_difference(name):
    q = Q.ALL[name]
    n = 18
    rng = np.random.default_rng(hash(name) % 1000)
    s, d = rand_graph(n, 110, 21)
    G = oracle.Graph(n, s, d)
    for step in range(6):
        before = brute.as_set(oracle.run(G, q, collect=True)["rows"])
        b = int(rng.integers(1, 25))
        bs = rng.integers(0, n, b).astype(np.uint32)
        bd = rng.integers(0, n, b).astype(np.uint32)
        sg = np.where(rng.random(b) < 0.4, -1, 1).astype(np.int8)
        # deletions target existing edges half of the time
        es, ed = G.edge_list()
        for k in range(b):
            if sg[k] < 0 and rng.random() < 0.5 and len(es):
                j = rng.integers(0, len(es))
                bs[k], bd[k] = es[j], ed[j]
        # drop insert/delete conflicts
        dels = {(int(x), int(y)) for x, y, g in zip(bs, bd, sg) if g < 0}
        keep = np.array([not (g > 0 and (int(x), int(y)) in dels) for x, y, g in zip(bs, bd, sg)])
        bs, bd, sg = bs[keep], bd[keep], sg[keep]
        r = oracle.delta(G, bs, bd, sg, q)
        after_rows = oracle.run(G, q, collect=True)["rows"]
        after = brute.as_set(after_rows)
        # the new graph equals the brute-force application of the batch
        A = brute.adjacency(n, *G.edge_list())
        assert brute.as_set(brute.matches(A, q)) == after
        got_plus = {t for t, g in zip(map(tuple, r["rows"].tolist()), r["signs"]) if g > 0}
        got_minus = {t for t, g in zip(map(tuple, r["rows"].tolist()), r["signs"]) if g < 0}
        assert got_plus == after - before
        assert got_minus == before - after
        assert r["count_delta"] == len(after) - len(before)
        assert set(np.unique(r["signs"]).tolist()) <= {-1, 1}


def test_delta_conflict_rejected():
    G = oracle.Graph(5, [0, 1], [1, 2])
    with pytest.raises(oracle.OracleError):
        oracle.delta(G, [3, 3], [4, 4], [1, -1], Q.TRIANGLE)
    assert G.num_edges == 2


def test_delta_noops_counted():
    G = oracle.Graph(5, [0, 1], [1, 2])
    oracle.delta(G, [0, 3, 4], [1, 4, 4], [1, -1, 1], Q.TRIANGLE)
    assert G.noops() == (1, 1)
    assert G.num_edges == 2


# ---------------------------------------------------------------- symmetry breaking (Sec. 5.4)
def rand_less(rng, m):
    pairs = [(x, y) for x in range(m) for y in range(m) if x != y]
    k = int(rng.integers(1, 4))
    return [pairs[i] for i in rng.choice(len(pairs), k, replace=False)]


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond",
                                  "cycle4", "reciprocal"])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_inequalities_brute_force(name, seed):
    """Inequality filters (Sec. 5.4) on random digraphs, random inequality sets
    and every valid order: the rows are the brute-force matches that satisfy
    the inequalities, and the extension counters do not depend on them."""
    rng = np.random.default_rng(100 + seed)
    q = Q.ALL[name]
    n = 8
    s, d = rand_graph(n, 30, 40 + seed)
    G = oracle.Graph(n, s, d)
    A = brute.adjacency(n, s, d)
    for order in Q.valid_orders(q)[:6]:
        less = rand_less(rng, q[0])
        ql = Q.with_less(Q.with_order(q, order), less)
        r = oracle.run(G, ql, collect=True)
        want = brute.matches(A, ql)
        assert brute.as_set(r["rows"]) == brute.as_set(want) and len(r["rows"]) == len(want)
        assert r["prefixes"][q[0]] == r["matches"] == len(want)
        plain = oracle.run(G, Q.with_order(q, order))
        assert r["extensions"][:2] == plain["extensions"][:2]
        assert r["prefixes"][2] <= plain["prefixes"][2]


def undirected_graph(n, m, seed):
    s, d = rand_graph(n, m, seed, loops=False)
    return oracle.symmetric_edges(n, s, d)


@pytest.mark.parametrize("name", sorted(Q.SYM_LESS))
def test_automorphism_identity(name):
    """On an undirected input the plain count is |Aut| times the count with
    the symmetry-breaking inequalities, in every valid order (each inequality
    is between adjacent attributes, so the group acts freely on matches)."""
    q = Q.ALL[name]
    less, aut = Q.SYM_LESS[name]
    n = 40 if q[0] < 5 else 18
    u, v = undirected_graph(n, 260 if q[0] < 5 else 160, 7)
    G = oracle.Graph(n, u, v)
    plain = oracle.run(G, q)["matches"]
    assert plain > 0
    for order in Q.valid_orders(q)[::7][:4]:
        sym = oracle.run(G, Q.with_less(Q.with_order(q, order), less))["matches"]
        assert sym * aut == plain, order


def test_inequality_closed_form_complete_graph():
    """Complete undirected graph K_n: cliques with a1 < ... < ak number C(n, k);
    the plain clique count is n! / (n - k)!."""
    n = 9
    s, d = np.nonzero(~np.eye(n, dtype=bool))
    G = oracle.Graph(n, s, d)
    for name, k in (("triangle", 3), ("clique4", 4), ("clique5", 5)):
        q = Q.ALL[name]
        less = [(i, i + 1) for i in range(k - 1)]
        assert oracle.run(G, Q.with_less(q, less))["matches"] == math.comb(n, k)
        assert oracle.run(G, q)["matches"] == math.perm(n, k)
        # contradictory inequalities leave nothing
        assert oracle.run(G, Q.with_less(q, [(0, 1), (1, 0)]))["matches"] == 0


@pytest.mark.parametrize("name", ["triangle", "clique4", "house"])
def test_delta_with_inequalities_equals_recompute_difference(name):
    """Delta-GJ of a query with inequalities: the signed rows are exactly the
    change of the static result."""
    q = Q.with_less(Q.ALL[name], Q.SYM_LESS[name][0])
    n = 12
    rng = np.random.default_rng(5)
    u, v = undirected_graph(n, 50, 9)
    G = oracle.Graph(n, u, v)
    for step in range(5):
        before = brute.as_set(oracle.run(G, q, collect=True)["rows"])
        b = int(rng.integers(1, 20))
        bs = rng.integers(0, n, b).astype(np.uint32)
        bd = rng.integers(0, n, b).astype(np.uint32)
        sg = np.where(rng.random(b) < 0.4, -1, 1).astype(np.int8)
        dels = {(int(x), int(y)) for x, y, g in zip(bs, bd, sg) if g < 0}
        keep = np.array([not (g > 0 and (int(x), int(y)) in dels) for x, y, g in zip(bs, bd, sg)])
        r = oracle.delta(G, bs[keep], bd[keep], sg[keep], q)
        after = brute.as_set(brute.matches(brute.adjacency(n, *G.edge_list()), q))
        assert brute.as_set(oracle.run(G, q, collect=True)["rows"]) == after
        plus = {t for t, g in zip(map(tuple, r["rows"].tolist()), r["signs"]) if g > 0}
        minus = {t for t, g in zip(map(tuple, r["rows"].tolist()), r["signs"]) if g < 0}
        assert plus == after - before and minus == before - after


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_degree_relabel_invariants(seed):
    """The renaming of Sec. 5.4: a permutation under which degrees ascend (ties
    by old id); the renamed edges are the input's distinct undirected pairs,
    once from the lower new id to the higher, or both ways."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 60))
    s, d = rand_graph(n, int(rng.integers(0, 4 * n)), 300 + seed)  # loops, repeats, reciprocal pairs
    pairs = {(min(a, b), max(a, b)) for a, b in zip(s.tolist(), d.tolist()) if a != b}
    deg = np.zeros(n, dtype=np.int64)
    for a, b in pairs:
        deg[a] += 1
        deg[b] += 1
    for undirected in (False, True):
        u, v, old = oracle.relabel_by_degree(n, s, d, undirected=undirected)
        assert sorted(old.tolist()) == list(range(n))
        key = [(int(deg[o]), int(o)) for o in old]
        assert key == sorted(key)
        back = {(min(int(old[a]), int(old[b])), max(int(old[a]), int(old[b]))) for a, b in zip(u, v)}
        assert back == pairs
        e = list(zip(u.tolist(), v.tolist()))
        assert e == sorted(set(e))
        if undirected:
            assert len(e) == 2 * len(pairs) and set(e) == {(b, a) for a, b in e}
        else:
            assert len(e) == len(pairs) and all(a < b for a, b in e)


def test_degree_relabel_star_and_clique_counts():
    """A star's centre has the largest degree, so it gets the last id and every
    edge points into it.  On a random undirected graph the plain clique query
    over the oriented graph counts each undirected clique once: the number of
    vertex subsets that are cliques, and the symmetric count over |Aut|."""
    import itertools
    k = 7
    s = np.full(k, 3, dtype=np.uint32)
    d = np.array([0, 1, 2, 4, 5, 6, 7], dtype=np.uint32)
    u, v, old = oracle.relabel_by_degree(k + 1, s, d)
    assert old[-1] == 3 and np.all(v == k) and len(u) == k
    n = 20
    a, b = undirected_graph(n, 110, 13)
    A = brute.adjacency(n, a, b)
    u, v, old = oracle.relabel_by_degree(n, a, b)
    G_or = oracle.Graph(n, u, v)
    G_sym = oracle.Graph(n, a, b)
    for name, kk in (("triangle", 3), ("clique4", 4), ("clique5", 5)):
        subsets = sum(all(A[x, y] for x, y in itertools.combinations(c, 2))
                      for c in itertools.combinations(range(n), kk))
        assert oracle.run(G_or, Q.ALL[name])["matches"] == subsets
        assert oracle.run(G_sym, Q.ALL[name])["matches"] == subsets * math.factorial(kk)


def test_invalid_inequalities():
    q = Q.TRIANGLE
    assert oracle.query_valid(Q.with_less(q, [(0, 2)]))
    assert not oracle.query_valid(Q.with_less(q, [(0, 0)]))
    assert not oracle.query_valid(Q.with_less(q, [(0, 3)]))


# ---------------------------------------------------------------- factorised counts (Sec. 5.4)
@pytest.mark.parametrize("name", sorted(Q.FACTORISABLE))
@pytest.mark.parametrize("seed", [0, 1])
def test_factorised_counts(name, seed):
    """Counting a trailing run of independent attributes as a product gives
    the plain count (and the brute-force one) in every order, with and without
    an inequality; counters up to the run are the plain ones, the run's
    prefixes are not materialised, and the extensions of each trailing
    attribute equal the plain count's extensions at the run's start in the
    order that binds that attribute first."""
    rng = np.random.default_rng(seed)
    q0 = Q.FACTORISABLE[name]
    n = 9
    s, d = rand_graph(n, 40, 500 + seed)
    G = oracle.Graph(n, s, d)
    A = brute.adjacency(n, s, d)
    m = q0[0]
    checked = 0
    for order in Q.valid_orders(q0)[::3]:
        for less in ([], rand_less(rng, m)[:1]):
            q = Q.with_less(Q.with_order(q0, order), less)
            f = oracle.run(G, q, factorise=True)
            p = oracle.run(G, q)
            assert f["matches"] == p["matches"] == len(brute.matches(A, q))
            j0 = Q.trailing_run(q)
            if not j0:
                assert f == p
                continue
            checked += 1
            assert f["prefixes"][:j0 + 1] == p["prefixes"][:j0 + 1]
            assert f["extensions"][:j0] == p["extensions"][:j0]
            assert f["prefixes"][j0 + 1:m] == [0] * (m - j0 - 1) and f["prefixes"][m] == f["matches"]
            for t in range(j0, m):
                o2 = list(order[:j0]) + [order[t]] + [order[u] for u in range(j0, m) if u != t]
                p2 = oracle.run(G, Q.with_less(Q.with_order(q0, o2), less))
                assert f["extensions"][t] == p2["extensions"][j0], (order, t)
    assert checked > 0


def test_factorised_closed_forms():
    """3-star: sum of out-degree cubes; fan: sum of in-degree times squared
    out-degree (join semantics: the leaves may coincide)."""
    n = 60
    s, d = rand_graph(n, 500, 77)
    G = oracle.Graph(n, s, d)
    es, ed = G.edge_list()
    out = np.bincount(es.astype(np.int64), minlength=n)
    inn = np.bincount(ed.astype(np.int64), minlength=n)
    assert oracle.run(G, Q.STAR3, factorise=True)["matches"] == int((out ** 3).sum())
    assert oracle.run(G, Q.FAN, factorise=True)["matches"] == int((inn * out ** 2).sum())


# ---------------------------------------------------------------- ternary atoms (Sec. 5.4)
@pytest.mark.parametrize("name", sorted(Q.TRI))
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_tri_atoms_brute_force(name, seed):
    """Queries over the triangle relation: rows equal the brute-force matches
    (tri(x, y, z) read as the three edges), with and without an inequality."""
    q = Q.TRI[name]
    n = 8 if q[0] < 5 else 7
    s, d = rand_graph(n, 36, 600 + seed)
    G = oracle.Graph(n, s, d)
    A = brute.adjacency(n, s, d)
    for less in ([], [(0, 2)]):
        ql = (q[0], q[1], q[2], less, q[4])
        r = oracle.run(G, ql, collect=True)
        want = brute.matches(A, ql)
        assert brute.as_set(r["rows"]) == brute.as_set(want) and len(r["rows"]) == len(want)


def test_tri_clique_identities():
    """The 4- and 5-clique over tri atoms count what the plain cliques count;
    the 4-clique's third position has as many prefixes, and its stage-2
    proposals sum |out(x) & out(y)| over the edges, both the plain triangle
    count."""
    n = 40
    s, d = rand_graph(n, 400, 31)
    G = oracle.Graph(n, s, d)
    tri = oracle.run(G, Q.TRIANGLE)["matches"]
    t4 = oracle.run(G, Q.TRI_CLIQUE4)
    assert t4["matches"] == oracle.run(G, Q.CLIQUE4)["matches"] > 0
    assert t4["prefixes"][3] == t4["extensions"][2] == tri
    assert oracle.run(G, Q.TRI_CLIQUE5)["matches"] == oracle.run(G, Q.CLIQUE5)["matches"]


def test_tri_complete_digraph():
    """Complete digraph K_n: every pair has n - 2 common out-neighbours."""
    n = 9
    s, d = np.nonzero(~np.eye(n, dtype=bool))
    G = oracle.Graph(n, s, d)
    r = oracle.run(G, Q.TRI_CLIQUE4)
    assert r["matches"] == n * (n - 1) * (n - 2) * (n - 3)
    assert r["extensions"][2] == n * (n - 1) * (n - 2)
    assert r["extensions"][3] == n * (n - 1) * (n - 2) * (n - 2)


def test_tri_invalid():
    assert oracle.query_valid(Q.TRI_CLIQUE4)
    assert not oracle.query_valid((3, [(0, 1)], [0, 1, 2], [], [(0, 2, 1)]))  # binds a middle attribute
    assert not oracle.query_valid((3, [(0, 1)], [0, 1, 2], [], [(0, 0, 2)]))
    assert not oracle.query_valid((3, [(0, 1)], [0, 1, 2], [], [(0, 1, 3)]))


@pytest.mark.parametrize("n", [4, 7, 10])
def test_counter_closed_forms(n):
    """Per-stage counters beyond the first stage, from closed forms (triangle,
    4-clique, 5-clique, diamond, 4-cycle).
    Complete digraph K_n: every set has n - 1 values, so each stage proposes
    n - 1 per prefix; prefixes are the tuples of the shape's distinctness.
    Transitive tournament (i -> j iff i < j): out(v) = n - 1 - v, so the
    smallest set of a prefix is the out-list of its largest vertex."""
    G = oracle.Graph(n, *complete(n))
    k = n - 1
    r = oracle.run(G, Q.TRIANGLE)
    assert r["prefixes"][2:4] == [n * k, n * k * (n - 2)] and r["extensions"][2] == n * k * k
    r = oracle.run(G, Q.CLIQUE4)
    assert r["prefixes"][3] == n * k * (n - 2) and r["extensions"][3] == n * k * (n - 2) * k
    r = oracle.run(G, Q.CLIQUE5)
    p4 = n * k * (n - 2) * (n - 3)
    assert r["prefixes"][4] == p4 and r["extensions"][4] == p4 * k and r["matches"] == p4 * (n - 4)
    for q in (Q.DIAMOND, Q.CYCLE4):  # a2 may repeat a1 (diamond) or a0 (4-cycle)
        r = oracle.run(G, q)
        assert r["prefixes"][3] == n * k * k and r["extensions"][2] == n * k * k
        assert r["extensions"][3] == n * k ** 3
    T = oracle.Graph(n, *tournament(n))
    r = oracle.run(T, Q.TRIANGLE)
    assert r["extensions"][2] == sum(j * (n - 1 - j) for j in range(n))
    r = oracle.run(T, Q.CLIQUE4)
    assert r["prefixes"][3] == math.comb(n, 3)
    assert r["extensions"][3] == sum(math.comb(z, 2) * (n - 1 - z) for z in range(n))
    r = oracle.run(T, Q.CLIQUE5)  # increasing tuples; the largest bound vertex has the shortest out-list
    assert r["prefixes"][4] == math.comb(n, 4) and r["matches"] == math.comb(n, 5)
    assert r["extensions"][4] == sum(math.comb(z, 3) * (n - 1 - z) for z in range(n))
