"""Pins of the oracle's 2-path closed form (diamond and 4-cycle counts with
their Generic Join counters) and of its incremental, threaded, count-only
Delta-GJ.  Every expected value here comes from an independent route: brute
force over vertex tuples, plain Python loops over the counters' definitions,
dense matrix identities, closed forms on the complete digraph, or numpy set
algebra for the effect of a batch.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from tests import brute
from tests import queries as Q


def rand_digraph(n, m, seed):
    rng = np.random.default_rng(seed)
    s = rng.integers(0, n, m).astype(np.uint32)
    d = rng.integers(0, n, m).astype(np.uint32)
    return s, d


def counters_by_definition(A, kind):
    """Generic Join counters of the order a0, a1, a2, a3, summed over the
    prefixes by plain loops: P_2 = edges; for the diamond a2 ranges over
    out(a0) and a3 is proposed from the smaller of out(a1), out(a2); for the
    4-cycle a2 ranges over out(a1) and a3 from the smaller of out(a2),
    in(a0)."""
    n = A.shape[0]
    outd = A.sum(axis=1)
    ind = A.sum(axis=0)
    E = [(u, v) for u in range(n) for v in range(n) if A[u, v]]
    pre3 = ext3 = 0
    for a0, a1 in E:
        if kind == "diamond":
            for a2 in range(n):
                if A[a0, a2]:
                    pre3 += 1
                    ext3 += min(outd[a1], outd[a2])
        else:
            for a2 in range(n):
                if A[a1, a2]:
                    pre3 += 1
                    ext3 += min(outd[a2], ind[a0])
    return len(E), pre3, ext3


@pytest.mark.parametrize("kind,query", [("diamond", Q.DIAMOND), ("cycle4", Q.CYCLE4)])
@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_twopath_brute_force_and_counters(kind, query, seed):
    """Random digraphs with unequal in- and out-degrees (so a swapped
    direction in any counter shows): count by brute force over all 4-tuples,
    counters by plain loops over the prefixes; the Generic Join oracle's
    counters agree with both."""
    n = 9
    s, d = rand_digraph(n, 34, 100 + seed)
    A = brute.adjacency(n, s, d)
    G = oracle.Graph(n, s, d)
    tp = oracle.twopath(G, kind, threads=1 + seed)
    assert tp["matches"] == len(brute.matches(A, query))
    e, pre3, ext3 = counters_by_definition(A, kind)
    assert tp["prefixes"][2] == e and tp["prefixes"][3] == pre3 and tp["extensions"][2] == pre3
    assert tp["extensions"][3] == ext3
    assert tp["prefixes"][4] == tp["matches"]
    gj = oracle.run(G, query)
    assert gj["matches"] == tp["matches"]
    assert gj["prefixes"][:5] == tp["prefixes"][:5]
    assert gj["extensions"][:5] == tp["extensions"][:5]


def test_twopath_counter_direction_matters():
    """A graph where |in(a0)| and |out(a0)| differ at every vertex that ends
    a 2-path: the 4-cycle's stage-3 counter with in(a0) replaced by out(a0)
    would give another value."""
    # the 4-cycles 0 -> 1 -> 2 -> 3 -> 0 and 0 -> 4 -> 2 -> 3 -> 0, extra
    # in-edges 5 -> 0, 6 -> 0
    s = np.array([0, 1, 2, 3, 0, 4, 5, 6], np.uint32)
    d = np.array([1, 2, 3, 0, 4, 2, 0, 0], np.uint32)
    A = brute.adjacency(7, s, d)
    G = oracle.Graph(7, s, d)
    tp = oracle.twopath(G, "cycle4")
    _, _, ext3 = counters_by_definition(A, "cycle4")
    swapped = sum(min(A[a2].sum(), A[a0].sum()) for a0 in range(7) for a1 in range(7) for a2 in range(7)
                  if A[a0, a1] and A[a1, a2])
    assert tp["extensions"][3] == ext3 != swapped
    # two 4-cycles, each in its four rotations
    assert tp["matches"] == len(brute.matches(A, Q.CYCLE4)) == 8


def test_twopath_er2000_dense_identities():
    """ER digraph n = 2,000, 20,000 arcs, seed 0: diamond = sum((A^2)^2),
    4-cycle = tr(A^4); prefixes[3] = sum_v out(v)^2 (diamond) and
    sum_v in(v) out(v) (4-cycle)."""
    s, d = synth.er_edges(2000, 20000, 0)
    A = brute.adjacency(2000, s, d).astype(np.float64)
    A2 = A @ A
    G = oracle.Graph(2000, s, d)
    dm = oracle.twopath(G, "diamond", threads=4)
    c4 = oracle.twopath(G, "cycle4", threads=4)
    assert dm["matches"] == int((A2 * A2).sum())
    assert c4["matches"] == int(np.trace(A2 @ A2))
    outd = A.sum(axis=1).astype(np.int64)
    ind = A.sum(axis=0).astype(np.int64)
    assert dm["prefixes"][3] == int((outd * outd).sum())
    assert c4["prefixes"][3] == int((outd * ind).sum())
    # and the Generic Join oracle's counters on the same graph
    for tp, q in ((dm, Q.DIAMOND), (c4, Q.CYCLE4)):
        r = oracle.run(G, q, threads=4)
        assert (r["matches"], r["prefixes"][:5], r["extensions"][:5]) == \
            (tp["matches"], tp["prefixes"][:5], tp["extensions"][:5])


@pytest.mark.parametrize("n", [2, 3, 6, 11])
def test_twopath_complete_digraph(n):
    """Complete digraph (every ordered pair, no loops): 2-paths a0 -> a3
    number n - 2 for a0 != a3 and n - 1 for a0 = a3, so the diamond counts
    n(n-1)(n-2)^2 + n(n-1)^2; the 4-cycle is tr((J - I)^4) =
    (n-1)^4 + (n-1)."""
    u, v = np.meshgrid(np.arange(n), np.arange(n))
    keep = u != v
    G = oracle.Graph(n, u[keep].astype(np.uint32), v[keep].astype(np.uint32))
    assert oracle.twopath(G, "diamond")["matches"] == n * (n - 1) * (n - 2) ** 2 + n * (n - 1) ** 2
    assert oracle.twopath(G, "cycle4")["matches"] == (n - 1) ** 4 + (n - 1)


def test_twopath_rmat_threads_and_gj():
    """R-MAT scale 10: any thread count gives the same result, equal to the
    Generic Join oracle's counts and counters."""
    s, d = synth.rmat_draws(10, seed=6)
    G = oracle.Graph(1 << 10, s, d)
    for kind, q in (("diamond", Q.DIAMOND), ("cycle4", Q.CYCLE4)):
        a = oracle.twopath(G, kind, threads=1)
        assert oracle.twopath(G, kind, threads=7) == a
        r = oracle.run(G, q, threads=4)
        assert (r["matches"], r["prefixes"][:5], r["extensions"][:5]) == \
            (a["matches"], a["prefixes"][:5], a["extensions"][:5])


# ---------------------------------------------------------------- Delta-GJ modes
def batches(n, count, seed, size=30):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        b = int(rng.integers(1, size))
        bs = rng.integers(0, n, b).astype(np.uint32)
        bd = rng.integers(0, n, b).astype(np.uint32)
        sg = np.where(rng.random(b) < 0.35, -1, 1).astype(np.int8)
        dels = {(int(x), int(y)) for x, y, g in zip(bs, bd, sg) if g < 0}
        keep = np.array([not (g > 0 and (int(x), int(y)) in dels) for x, y, g in zip(bs, bd, sg)])
        yield bs[keep], bd[keep], sg[keep]


@pytest.mark.parametrize("name", ["triangle", "clique4", "diamond", "cycle4", "reciprocal"])
def test_delta_count_only_and_threads(name):
    """The count-only mode returns the signed sum of the rows mode, the same
    emissions and counters; any thread count returns the same rows."""
    q = Q.ALL[name]
    n = 24
    s, d = rand_digraph(n, 160, 5)
    Ga, Gb, Gc = oracle.Graph(n, s, d), oracle.Graph(n, s, d), oracle.Graph(n, s, d)
    for bs, bd, sg in batches(n, 8, 9):
        ra = oracle.delta(Ga, bs, bd, sg, q, rows=True, threads=1)
        rb = oracle.delta(Gb, bs, bd, sg, q, rows=False, threads=3)
        rc = oracle.delta(Gc, bs, bd, sg, q, rows=True, threads=5)
        assert ra["count_delta"] == int(ra["signs"].astype(np.int64).sum()) == rb["count_delta"]
        assert ra["raw_emissions"] == rb["raw_emissions"] == rc["raw_emissions"]
        assert ra["prefixes"] == rb["prefixes"] == rc["prefixes"]
        assert ra["extensions"] == rb["extensions"] == rc["extensions"]
        assert np.array_equal(ra["rows"], rc["rows"]) and np.array_equal(ra["signs"], rc["signs"])
        assert "rows" not in rb


def test_delta_long_stream_incremental_state():
    """Sixty batches applied incrementally: after every batch the edge list
    equals the batch semantics applied with numpy set algebra (no-ops
    ignored, self-loops dropped), and at the end the static count has moved
    by the sum of the count deltas."""
    n = 1 << 8
    s, d = synth.rmat_draws(8, seed=2)
    G = oracle.Graph(n, s, d)
    key = lambda a, b: (np.asarray(a, np.int64) << 20) | np.asarray(b, np.int64)
    keys = np.unique(key(s, d)[s != d])
    c0 = oracle.run(G, Q.TRIANGLE)["matches"]
    total = 0
    for bs, bd, sg in batches(n, 60, 4, size=120):
        # deletions of present edges
        es, ed = G.edge_list()
        rng = np.random.default_rng(len(bs))
        for k in range(len(bs)):
            if sg[k] < 0 and len(es):
                j = int(rng.integers(0, len(es)))
                bs[k], bd[k] = es[j], ed[j]
        dels = {(int(x), int(y)) for x, y, g in zip(bs, bd, sg) if g < 0}
        keep = np.array([not (g > 0 and (int(x), int(y)) in dels) for x, y, g in zip(bs, bd, sg)], bool)
        bs, bd, sg = bs[keep], bd[keep], sg[keep]
        r = oracle.delta(G, bs, bd, sg, Q.TRIANGLE, rows=False, threads=2)
        total += r["count_delta"]
        bk = key(bs, bd)
        loops = bs == bd
        keys = np.union1d(np.setdiff1d(keys, bk[(sg < 0) & ~loops]), bk[(sg > 0) & ~loops])
        es, ed = G.edge_list()
        assert np.array_equal(key(es, ed), keys)
        assert G.num_edges == len(keys)
    assert oracle.run(G, Q.TRIANGLE)["matches"] - c0 == total
