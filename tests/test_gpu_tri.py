"""GPU parity of ternary atoms over the triangle relation (Sec. 5.4) against
the CPU oracle, which evaluates tri(x, y, z) from its definition: the index
itself (a query with one tri atom lists every transitive triangle), the
4- and 5-clique rewrites and a mixed query (counts, counters, rows), index
builds split into many chunks, staleness after updates, and the paths that
reject such queries."""
import numpy as np
import pytest

import oracle
import synth
from tests import queries as Q

pytestmark = pytest.mark.gpu

ONE_TRI = (3, [(0, 1)], [0, 1, 2], [], [(0, 1, 2)])


@pytest.fixture(scope="module")
def gj():
    import paper_1802_03760_amd as gj
    return gj


def gq(gj, ctx, q):
    return gj.Query(ctx, q[0], q[1], q[2], less=q[3] if len(q) > 3 else (), tris=q[4] if len(q) > 4 else ())


def check(gj, ctx, G, O, q, enumerate_=True):
    ref = oracle.run(O, q, collect=enumerate_, threads=8)
    h = gq(gj, ctx, q)
    r = gj.count(ctx, G, h)
    assert (r["matches"], r["prefixes"], r["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"]), q
    if enumerate_:
        st, rows = gj.enumerate_rows(ctx, G, h)
        assert np.array_equal(np.asarray(rows), ref["rows"]), q
    return ref


@pytest.mark.parametrize("opts", [{}, {"seed_chunk": 500, "frontier_cap": 64}])
def test_index_and_rewrites(gj, opts):
    c = gj.Context(0)
    for k, v in opts.items():
        c.set_option(k, v)
    src, dst = synth.rmat_draws(10, seed=31)
    n = 1 << 10
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    ntri = G.index_triangles()
    ref = check(gj, c, G, O, ONE_TRI)
    assert ntri == ref["matches"] == oracle.run(O, Q.TRIANGLE)["matches"]
    # the index lists the plain triangle query's rows, edge by edge
    assert np.array_equal(gj.enumerate_rows(c, G, gj.Query(c, *Q.TRIANGLE))[1], ref["rows"])
    for name, q in sorted(Q.TRI.items()):
        check(gj, c, G, O, q, enumerate_=name != "tri_clique5")
        check(gj, c, G, O, (q[0], q[1], q[2], [(1, 2)], q[4]), enumerate_=False)
    assert gj.count(c, G, gq(gj, c, Q.TRI_CLIQUE4))["matches"] == gj.count(c, G, gj.Query(c, *Q.CLIQUE4))["matches"]


def test_stale_after_update_and_rejections(gj):
    c = gj.Context(0)
    src, dst = synth.rmat_draws(9, seed=32)
    n = 1 << 9
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    h = gq(gj, c, Q.TRI_CLIQUE4)
    with pytest.raises(gj.GJError):  # no index yet
        gj.count(c, G, h)
    G.index_triangles()
    check(gj, c, G, O, Q.TRI_CLIQUE4, enumerate_=False)
    with pytest.raises(gj.GJError):
        gj.run_batch(c, G, [(h, 0, 100)])
    with pytest.raises(gj.GJError):
        gj.apply_updates(c, G, np.array([1], np.uint32), np.array([2], np.uint32), np.array([1], np.int8), [h])
    S = gj.Server(c, G)
    with pytest.raises(gj.GJError):
        S.submit_count(h)
    S.close()
    for k, bs, bd, bg in synth.update_stream(9, 32, 33, 2, 1, 200):
        gj.apply_updates(c, G, bs, bd, bg, [])
        oracle.delta(O, bs, bd, bg)
    with pytest.raises(gj.GJError):  # stale
        gj.count(c, G, h)
    G.index_triangles()
    check(gj, c, G, O, Q.TRI_CLIQUE4)


def test_empty_and_errors(gj):
    c = gj.Context(0)
    G = gj.Graph(c, np.array([], np.uint32), np.array([], np.uint32), 4)
    assert G.index_triangles() == 0
    assert gj.count(c, G, gq(gj, c, Q.TRI_CLIQUE4))["matches"] == 0
    G2 = gj.Graph(c, np.array([0, 1], np.uint32), np.array([1, 2], np.uint32), 3)
    assert G2.index_triangles() == 0
    for bad in ((3, [(0, 1)], [0, 1, 2], [], [(0, 2, 1)]), (3, [(0, 1)], [0, 1, 2], [], [(0, 0, 2)]),
                (3, [(0, 1)], [0, 1, 2], [], [(0, 1, 3)])):
        with pytest.raises(gj.GJError):
            gq(gj, c, bad)
