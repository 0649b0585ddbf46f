"""GPU parity of the static Generic Join path (gj_run through the C ABI)
against the CPU oracle: bit-exact counts, per-stage counters and sorted
match lists."""
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


def check(gj, ctx, n, src, dst, q, enumerate_=True, seed_lo=0, seed_hi=None, G=None, O=None):
    G = G or gj.Graph(ctx, src, dst, n)
    O = O or oracle.Graph(n, src, dst)
    hi = (1 << 64) - 1 if seed_hi is None else seed_hi
    ref = oracle.run(O, q, collect=enumerate_, seed_lo=seed_lo, seed_hi=seed_hi, threads=4)
    Qh = gj.Query(ctx, q[0], q[1], q[2])
    c = gj.count(ctx, G, Qh, seed_lo, hi)
    assert c["matches"] == ref["matches"], (q, c["matches"], ref["matches"])
    assert c["prefixes"] == ref["prefixes"], (c["prefixes"], ref["prefixes"])
    assert c["extensions"] == ref["extensions"], (c["extensions"], ref["extensions"])
    if enumerate_:
        st, rows = gj.enumerate_rows(ctx, G, Qh, seed_lo, hi)
        assert st["matches"] == ref["matches"]
        assert np.array_equal(np.asarray(rows), ref["rows"])
    return ref


def test_er2000_triangle(gj, ctx):
    """Directed triangle on the ER digraph: n = 2,000, 20,000 distinct arcs, seed 0."""
    src, dst = synth.er_edges(2000, 20000, 0)
    ref = check(gj, ctx, 2000, src, dst, Q.TRIANGLE)
    assert ref["matches"] > 0


@pytest.mark.parametrize("name", sorted(Q.ALL))
def test_small_random_all_orders(gj, ctx, name):
    q = Q.ALL[name]
    n = 40 if q[0] <= 4 else 16
    rng = np.random.default_rng(len(name))
    src = rng.integers(0, n, n * 8).astype(np.uint32)
    dst = rng.integers(0, n, n * 8).astype(np.uint32)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    orders = Q.valid_orders(q)
    for order in orders[:: max(1, len(orders) // 6)]:
        check(gj, ctx, n, src, dst, Q.with_order(q, order), G=G, O=O)


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4"])
def test_rmat12(gj, ctx, name):
    src, dst = synth.rmat_draws(12, seed=1)
    check(gj, ctx, 1 << 12, src, dst, Q.ALL[name], enumerate_=name in ("triangle", "clique4"))


def test_small_batches_force_deep_schedule(gj, ctx):
    """Tiny frontier and seed caps: many proposal batches per stage, ragged
    tails, depth-first recursion through every level."""
    src, dst = synth.rmat_draws(10, seed=2)
    n = 1 << 10
    c2 = gj.Context(0)
    c2.set_option("frontier_cap", 100)
    c2.set_option("seed_chunk", 37)
    for q in (Q.TRIANGLE, Q.CLIQUE4, Q.DIAMOND, Q.HOUSE):
        check(gj, c2, n, src, dst, q, enumerate_=q is not Q.DIAMOND)


def test_seed_slices(gj, ctx):
    src, dst = synth.rmat_draws(11, seed=3)
    n = 1 << 11
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    E = G.info()["edges"]
    assert E == O.num_edges
    for lo, hi in [(0, 1), (5, 900), (E // 3, E // 2), (E - 7, E), (E, E + 10), (0, E)]:
        check(gj, ctx, n, src, dst, Q.TRIANGLE, seed_lo=lo, seed_hi=hi, G=G, O=O)
        check(gj, ctx, n, src, dst, Q.CYCLIC_TRIANGLE, seed_lo=lo, seed_hi=hi, G=G, O=O)


def test_complete_digraph_closed_forms(gj, ctx):
    n = 9
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    src, dst = s[keep].astype(np.uint32), d[keep].astype(np.uint32)
    G = gj.Graph(ctx, src, dst, n)
    for q, want in [(Q.TRIANGLE, n * (n - 1) * (n - 2)), (Q.CLIQUE4, n * (n - 1) * (n - 2) * (n - 3)),
                    (Q.CLIQUE5, n * (n - 1) * (n - 2) * (n - 3) * (n - 4)),
                    (Q.HOUSE, n * (n - 1) * (n - 2) * (n - 3) * (n - 2)),
                    (Q.DIAMOND, (n - 1) ** 4 + (n - 1)), (Q.CYCLE4, (n - 1) ** 4 + (n - 1))]:
        assert gj.count(ctx, G, gj.Query(ctx, *q))["matches"] == want


def test_edge_cases(gj, ctx):
    # empty graph, only self-loops, one edge, duplicates
    for src, dst, n in [([], [], 5), ([1, 2, 3], [1, 2, 3], 4), ([0], [1], 2),
                        ([0, 0, 0, 1, 1, 2], [1, 1, 1, 2, 2, 0], 3)]:
        src = np.array(src, dtype=np.uint32)
        dst = np.array(dst, dtype=np.uint32)
        for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE, Q.RECIPROCAL, (2, [(0, 1)], [0, 1]), (2, [(0, 1)], [1, 0])):
            check(gj, ctx, n, src, dst, q)


def test_star_hub(gj, ctx):
    """One hub of degree 20,000 with reciprocal arcs to every leaf, leaves
    chained: skewed extension sets on both sides."""
    n = 20001
    leaves = np.arange(1, n, dtype=np.uint32)
    src = np.concatenate([np.zeros(n - 1, np.uint32), leaves, leaves[:-1]])
    dst = np.concatenate([leaves, np.zeros(n - 1, np.uint32), leaves[1:]])
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE, Q.DIAMOND):
        check(gj, ctx, n, src, dst, q, enumerate_=q is not Q.DIAMOND)


def test_csr_matches_edge_set(gj, ctx):
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    src, dst = synth.rmat_draws(11, seed=4)
    n = 1 << 11
    G = gj.Graph(ctx, src, dst, n)
    E = G.info()["edges"]
    es, ed = oracle.Graph(n, src, dst).edge_list()
    for rev in (0, 1):
        rp, col, row = G.csr_ptrs(rev)
        h_rp = np.empty(n + 1, np.uint32)
        h_col = np.empty(E, np.uint32)
        h_row = np.empty(E, np.uint32)
        for arr, p in ((h_rp, rp), (h_col, col), (h_row, row)):
            # hipMemcpyDeviceToHost = 2
            assert hip.hipMemcpy(ctypes.c_void_p(arr.ctypes.data), ctypes.c_void_p(p),
                                 ctypes.c_size_t(arr.nbytes), 2) == 0
        a, b = (es, ed) if rev == 0 else (ed, es)
        order = np.lexsort((b, a))
        assert np.array_equal(h_row, a[order]) and np.array_equal(h_col, b[order])
        assert np.array_equal(h_rp, np.searchsorted(a[order], np.arange(n + 1)).astype(np.uint32))


def test_errors(gj, ctx):
    with pytest.raises(gj.GJError) as e:
        gj.Graph(ctx, np.array([0, 9], np.uint32), np.array([1, 2], np.uint32), 5)
    assert e.value.status == gj.GJ_EINVAL
    for bad in [(3, [(0, 1), (1, 2)], [0, 2, 1]), (3, [(0, 0), (0, 1), (1, 2)], [0, 1, 2]),
                (4, [(0, 1), (2, 3)], [0, 1, 2, 3]), (3, [(0, 1), (1, 2)], [0, 1, 1])]:
        with pytest.raises(gj.GJError) as e:
            gj.Query(ctx, *bad)
        assert e.value.status == gj.GJ_EINVAL
    src, dst = synth.er_edges(200, 2000, 1)
    G = gj.Graph(ctx, src, dst, 200)
    q = gj.Query(ctx, *Q.TRIANGLE)
    n = gj.count(ctx, G, q)["matches"]
    assert n > 2
    with pytest.raises(gj.GJError) as e:
        gj.enumerate_rows(ctx, G, q, cap=n - 1)
    assert e.value.status == gj.GJ_EOVERFLOW


@pytest.mark.parametrize("cap", [64, 1 << 25])
def test_propose_widths_agree(gj, cap):
    """The generic propose kernel tests 1, 2 or 4 candidates per lane in
    lockstep; counts, counters and rows are the oracle's for every width,
    with frontier caps that make odd word counts and ragged wave runs."""
    src, dst = synth.rmat_draws(9, seed=41)
    n = 1 << 9
    O = oracle.Graph(n, src, dst)
    c = gj.Context(0)
    c.set_option("frontier_cap", cap)
    G = gj.Graph(c, src, dst, n)
    for q in (Q.CLIQUE4, Q.DIAMOND, Q.CYCLE4, Q.with_less(Q.HOUSE, [(1, 2)])):
        ref = oracle.run(O, q, collect=q[0] < 5, threads=8)
        h = gj.Query(c, *q)
        for u in (1, 2, 4):
            c.set_option("propose_u", u)
            r = gj.count(c, G, h)
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), (q, u)
            if q[0] < 5:
                assert np.array_equal(gj.enumerate_rows(c, G, h)[1], ref["rows"]), (q, u)
    with pytest.raises(gj.GJError):
        c.set_option("propose_u", 3)


def test_clique4_edge_grouped_kernel(gj, ctx):
    """Full 4-clique and diamond counts run grouped by seed edge; seeds whose
    fixed set exceeds the kernel's LDS share (1,024 entries) finish on the
    depth-first path.  Hub pairs with 300, 1,030 and 16,400 common
    neighbours (chained so 4-cliques exist) fall on both sides.  Counts and
    every counter equal the oracle's and the generic path's (strategy 1)."""
    s, d = [], []
    base = 0
    for k in (300, 1030, 16400):
        h0, h1 = base, base + 1
        common = np.arange(base + 2, base + 2 + k, dtype=np.uint32)
        s += [np.array([h0], np.uint32), np.full(k, h0, np.uint32), np.full(k, h1, np.uint32), common[:-1]]
        d += [np.array([h1], np.uint32), common, common, common[1:]]
        base += k + 2
    rs, rd = synth.rmat_draws(11, seed=44)  # an R-MAT background
    s.append(rs + base)
    d.append(rd + base)
    k = 300
    src, dst = np.concatenate(s), np.concatenate(d)
    n = base + (1 << 11)
    G, O = gj.Graph(ctx, src, dst, n), oracle.Graph(n, src, dst)
    c1 = gj.Context(0)
    c1.set_option("strategy", 1)
    G1 = gj.Graph(c1, src, dst, n)
    for q in (Q.CLIQUE4, Q.DIAMOND):
        ref = oracle.run(O, q, threads=8)
        assert ref["matches"] >= k - 1
        for cc, GG in ((ctx, G), (c1, G1)):
            r = gj.count(cc, GG, gj.Query(cc, *q))
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), q


def test_clique5_edge_grouped_kernel(gj, ctx):
    """Full transitive 5-clique counts run grouped by seed edge, with the
    common neighbourhood's adjacency as bit masks in LDS: a wave per seed up
    to 256 common neighbours, a workgroup up to 704, the depth-first path
    beyond.  Hub pairs with 200, 300 and 720 common neighbours (each joined
    to the next two, so that 5-cliques exist) take the three, over an R-MAT
    background.  Then the degree-ordered form, random inequality sets, and
    the symmetry-breaking set on the undirected form.  Counts and every
    counter equal the oracle's and the generic path's (strategy 1)."""
    from tests.test_gpu_sym import rand_less
    s, d = [], []
    base = 0
    for k in (200, 300, 720):
        h0, h1 = base, base + 1
        common = np.arange(base + 2, base + 2 + k, dtype=np.uint32)
        s += [np.array([h0], np.uint32), np.full(k, h0, np.uint32), np.full(k, h1, np.uint32),
              common[:-1], common[:-2]]
        d += [np.array([h1], np.uint32), common, common, common[1:], common[2:]]
        base += k + 2
    rs, rd = synth.rmat_draws(11, seed=45)
    s.append(rs + base)
    d.append(rd + base)
    src, dst = np.concatenate(s), np.concatenate(d)
    n = base + (1 << 11)
    c1 = gj.Context(0)
    c1.set_option("strategy", 1)

    def check(G, G1, O, q):
        ref = oracle.run(O, q, threads=8)
        for cc, GG in ((ctx, G), (c1, G1)):
            r = gj.count(cc, GG, gj.Query(cc, *q))
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), q
        return ref

    G, G1, O = gj.Graph(ctx, src, dst, n), gj.Graph(c1, src, dst, n), oracle.Graph(n, src, dst)
    ref = check(G, G1, O, Q.CLIQUE5)
    assert ref["matches"] >= 198 + 298 + 718
    rng = np.random.default_rng(5)
    for _ in range(3):
        check(G, G1, O, Q.with_less(Q.CLIQUE5, rand_less(rng, 5)))
    # degree-ordered: the oracle renames the same way
    Gd, Gd1 = gj.Graph(ctx, src, dst, n, degree_order=True), gj.Graph(c1, src, dst, n, degree_order=True)
    ds, dd, _ = oracle.relabel_by_degree(n, src, dst)
    check(Gd, Gd1, oracle.Graph(n, ds, dd), Q.CLIQUE5)
    # undirected with the symmetry-breaking chain a0 < a1 < a2 < a3 < a4
    u, v = oracle.symmetric_edges(n, src, dst)
    Gu, Gu1, Ou = (gj.Graph(ctx, src, dst, n, undirected=True), gj.Graph(c1, src, dst, n, undirected=True),
                   oracle.Graph(n, u, v))
    less, aut = Q.SYM_LESS["clique5"]
    refu = check(Gu, Gu1, Ou, Q.with_less(Q.CLIQUE5, less))
    assert gj.count(ctx, Gu, gj.Query(ctx, *Q.CLIQUE5))["matches"] == aut * refu["matches"]


def test_clique4_edge_grouped_inequalities(gj, ctx):
    """The edge-grouped 4-clique and diamond kernels with inequalities on a3
    (each a2's range of S and of its own row narrowed by binary search):
    hub pairs with 300, 1,030 and 16,400 common neighbours (the wave, the
    workgroup and the depth-first path) plus an R-MAT background, directed
    with several inequality sets and undirected with the symmetry-breaking
    order.  Counts and counters equal the oracle's and the generic path's."""
    s, d = [], []
    base = 0
    for k in (300, 1030, 16400):
        h0, h1 = base + k + 1, base  # one hub pair with the larger id first
        common = np.arange(base + 2, base + 2 + k, dtype=np.uint32)[::-1].copy()
        s += [np.array([h0], np.uint32), np.full(k, h0, np.uint32), np.full(k, h1, np.uint32), common[:-1],
              common[1:]]
        d += [np.array([h1], np.uint32), common, common, common[1:], common[:-1]]
        base += k + 2
    rs, rd = synth.rmat_draws(11, seed=45)
    s.append(rs + base)
    d.append(rd + base)
    src, dst = np.concatenate(s), np.concatenate(d)
    n = base + (1 << 11)
    c1 = gj.Context(0)
    c1.set_option("strategy", 1)
    cases = [(Q.CLIQUE4, [(0, 1), (1, 2), (2, 3)]), (Q.CLIQUE4, [(2, 3)]), (Q.CLIQUE4, [(3, 2)]),
             (Q.CLIQUE4, [(0, 3), (3, 1)]), (Q.CLIQUE4, [(3, 0), (2, 3)]),
             (Q.DIAMOND, [(0, 3), (3, 2)])]  # the diamond's oracle run alone takes about 12 s here
    G, O = gj.Graph(ctx, src, dst, n), oracle.Graph(n, src, dst)
    G1 = gj.Graph(c1, src, dst, n)
    for q, less in cases:
        qq = Q.with_less(q, less)
        ref = oracle.run(O, qq, threads=8)
        for cc, GG in ((ctx, G), (c1, G1)):
            r = gj.count(cc, GG, gj.Query(cc, *qq))
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), (q, less)
    u, v = oracle.symmetric_edges(n, src, dst)
    Gu, Ou = gj.Graph(ctx, src, dst, n, undirected=True), oracle.Graph(n, u, v)
    qq = Q.with_less(Q.CLIQUE4, Q.SYM_LESS["clique4"][0])
    ref = oracle.run(Ou, qq, threads=8)
    assert ref["matches"] > 0
    r = gj.count(ctx, Gu, gj.Query(ctx, *qq))
    assert (r["matches"], r["prefixes"], r["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"])
