"""Parity at full workload sizes, in the launch configuration bench.py times.

R-MAT scale 22 (65.2M edges) and scale 20 (16.1M edges): the full counts are
checked through properties that hold at any size (edge count and extension
counter computed independently with numpy; the owner-grouped count equals the
generic per-candidate count), and sampled seed slices are checked
element by element against the oracle.  Delta batches at scale 22 are
checked by count conservation, by validity of every reported row, and by the
largest degrees and row pointers of the new versions.
"""
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


def distinct_edges(src, dst):
    k = (src.astype(np.uint64) << np.uint64(32)) | dst.astype(np.uint64)
    k = np.unique(k[src != dst])
    return (k >> np.uint64(32)).astype(np.int64), (k & np.uint64(0xFFFFFFFF)).astype(np.int64)


def slices(E, count, width):
    return [((E * i) // count, min(E, (E * i) // count + width)) for i in range(count)]


@pytest.fixture(scope="module")
def rmat22(gj):
    src, dst = synth.rmat_draws(22, seed=0)
    return src, dst


@pytest.fixture(scope="module")
def oracle22(rmat22):
    src, dst = rmat22
    return oracle.Graph(1 << 22, src, dst)


def test_rmat22_triangle_count(gj, rmat22, oracle22):
    src, dst = rmat22
    n = 1 << 22
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    q = gj.Query(ctx, *Q.TRIANGLE)
    full = gj.count(ctx, G, q)  # owner-grouped kernel, as in bench.py
    assert full["kernel_launches"] == 1
    es, ed = distinct_edges(src, dst)
    assert full["prefixes"][2] == len(es) == G.info()["edges"]
    outd = np.bincount(es, minlength=n)
    assert full["extensions"][2] == int(np.minimum(outd[es], outd[ed]).sum())
    # Generic Join's work bound (Sec. 2.2; Chiba-Nishizeki: 2 a(G) |E|)
    E0 = len(es)
    assert full["extensions"][2] <= 2 * int(np.ceil(np.sqrt(2 * E0 + n) / 2)) * E0
    # generic per-candidate kernel on the same graph
    gen = gj.Context(0)
    gen.set_option("strategy", 1)
    G2 = gj.Graph(gen, src, dst, n)
    g = gj.count(gen, G2, gj.Query(gen, *Q.TRIANGLE))
    assert g["matches"] == full["matches"] and g["extensions"] == full["extensions"]
    # sampled seed slices: generic kernel vs oracle, element by element
    O = oracle22
    E = O.num_edges
    for lo, hi in slices(E, 8, 3000):
        ref = oracle.run(O, Q.TRIANGLE, collect=True, seed_lo=lo, seed_hi=hi, threads=16)
        st, rows = gj.enumerate_rows(gen, G2, gj.Query(gen, *Q.TRIANGLE), lo, hi)
        assert st["matches"] == ref["matches"] and np.array_equal(rows, ref["rows"]), (lo, hi)
        assert st["extensions"] == ref["extensions"]
    G2.close()
    gen.close()
    G.close()
    ctx.close()


def test_rmat22_four_clique_and_diamond_slices(gj, rmat22, oracle22):
    src, dst = rmat22
    n = 1 << 22
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle22
    E = O.num_edges
    for q, width in ((Q.CLIQUE4, 400), (Q.CYCLIC_TRIANGLE, 2000)):
        qh = gj.Query(ctx, *q)
        # the first slice starts at the hubs: 20 seeds there keep the oracle within seconds
        for lo, hi in [(0, 20)] + slices(E, 6, width)[1:]:
            ref = oracle.run(O, q, seed_lo=lo, seed_hi=hi, threads=16)
            got = gj.count(ctx, G, qh, lo, hi)
            assert got["matches"] == ref["matches"], (q, lo, hi)
            assert got["prefixes"] == ref["prefixes"] and got["extensions"] == ref["extensions"]
    # diamond: seeds from the low-degree end of the edge range
    qh = gj.Query(ctx, *Q.DIAMOND)
    for lo in (E - 5000, E - 40000):
        ref = oracle.run(O, Q.DIAMOND, seed_lo=lo, seed_hi=lo + 200, threads=16)
        got = gj.count(ctx, G, qh, lo, lo + 200)
        assert got["matches"] == ref["matches"] and got["extensions"] == ref["extensions"]
    G.close()
    ctx.close()


@pytest.mark.timeout(900)
def test_rmat20_full_sorted_enumeration(gj):
    """Every row of the R-MAT-20 triangle enumeration (570,418,567 sorted
    rows) against the oracle's, element by element, in 64 seed slices that
    cover the whole edge range; the slices' rows are each sorted and follow
    one another in order, so their concatenation is the full sorted
    enumeration, and its length is the whole count."""
    src, dst = synth.rmat_draws(20, seed=0)
    n = 1 << 20
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    E = O.num_edges
    q = gj.Query(ctx, *Q.TRIANGLE)
    full = gj.count(ctx, G, q)["matches"]
    total, prev = 0, None
    for i in range(64):
        lo, hi = E * i // 64, E * (i + 1) // 64
        ref = oracle.run(O, Q.TRIANGLE, collect=True, seed_lo=lo, seed_hi=hi, threads=16)
        st, rows = gj.enumerate_rows(ctx, G, q, lo, hi)
        assert st["matches"] == ref["matches"] and np.array_equal(rows, ref["rows"]), (i, lo, hi)
        if len(rows):
            if prev is not None:
                assert tuple(prev) < tuple(rows[0]), i  # slices follow one another in sorted order
            prev = rows[-1].copy()
        total += st["matches"]
        del ref, rows
    assert total == full == 570418567
    G.close()
    ctx.close()


def test_rmat20_enumerate_slices(gj):
    """R-MAT scale 20 triangle count and enumeration (sorted rows) on
    sampled seed slices; the full count through both kernels."""
    src, dst = synth.rmat_draws(20, seed=0)
    n = 1 << 20
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    E = O.num_edges
    q = gj.Query(ctx, *Q.TRIANGLE)
    full = gj.count(ctx, G, q)
    gen = gj.Context(0)
    gen.set_option("strategy", 1)
    G2 = gj.Graph(gen, src, dst, n)
    assert gj.count(gen, G2, gj.Query(gen, *Q.TRIANGLE))["matches"] == full["matches"]
    for lo, hi in slices(E, 10, 5000):
        ref = oracle.run(O, Q.TRIANGLE, collect=True, seed_lo=lo, seed_hi=hi, threads=16)
        st, rows = gj.enumerate_rows(ctx, G, q, lo, hi)
        assert np.array_equal(rows, ref["rows"]), (lo, hi)
    G2.close()
    gen.close()
    G.close()
    ctx.close()


def test_rmat22_delta_stream_properties(gj, rmat22):
    """Delta batches on the scale-22 graph: the sum of count deltas equals
    the change of the full count, and every reported row is a triangle of
    the new graph (sign +1) or of the old graph (sign -1), not of both."""
    src, dst = rmat22
    n = 1 << 22
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    q = gj.Query(ctx, *Q.TRIANGLE)
    c0 = gj.count(ctx, G, q)["matches"]
    es, ed = distinct_edges(src, dst)
    keys = np.sort((es << 32) | ed)
    total = 0
    for k, bs, bd, bg in synth.update_stream(22, 0, 1, 6, 1, 20000):
        r = gj.apply_updates(ctx, G, bs, bd, bg, [q], rows=True)[0]
        total += r["count_delta"]
        assert r["count_delta"] == int(r["signs"].astype(np.int64).sum())
        # the edge set after the batch, by numpy
        bk = (bs.astype(np.int64) << 32) | bd.astype(np.int64)
        loops = bs == bd
        ins = np.setdiff1d(bk[(bg > 0) & ~loops], keys)
        dels = np.intersect1d(bk[(bg < 0) & ~loops], keys)
        new_keys = np.union1d(np.setdiff1d(keys, dels), ins)
        info = G.info()
        assert info["edges"] == len(new_keys)
        deg_out = np.bincount((new_keys >> 32).astype(np.int64), minlength=n)
        deg_in = np.bincount((new_keys & 0xFFFFFFFF).astype(np.int64), minlength=n)
        assert (info["max_out"], info["max_in"]) == (int(deg_out.max()), int(deg_in.max()))
        rows = r["rows"].astype(np.int64)
        if len(rows):
            def present(kk, a, b):
                x = (a << 32) | b
                i = np.searchsorted(kk, x)
                return (i < len(kk)) & (kk[np.minimum(i, len(kk) - 1)] == x)

            def tri(kk):
                return (present(kk, rows[:, 0], rows[:, 1]) & present(kk, rows[:, 1], rows[:, 2])
                        & present(kk, rows[:, 0], rows[:, 2]))
            t_new, t_old = tri(new_keys), tri(keys)
            assert np.all(np.where(r["signs"] > 0, t_new & ~t_old, t_old & ~t_new))
        keys = new_keys
    c1 = gj.count(ctx, G, q)["matches"]
    assert c1 - c0 == total
    # row pointers of both directions of the last version
    hip = ctypes.CDLL("libamdhip64.so")
    for rev, deg in ((0, deg_out), (1, deg_in)):
        rp = np.empty(n + 1, np.uint32)
        assert hip.hipMemcpy(ctypes.c_void_p(rp.ctypes.data), ctypes.c_void_p(G.csr_ptrs(rev)[0]),
                             ctypes.c_size_t(rp.nbytes), 2) == 0
        assert rp[0] == 0 and np.array_equal(np.diff(rp.astype(np.int64)), deg), rev
    G.close()
    ctx.close()


def test_rmat22_factorised_closed_forms(gj, rmat22):
    """Factorised counts at scale 22 against closed forms computed with numpy:
    the 3-star counts sum out(v)^3 and the fan sum in(v) out(v)^2; the first
    trailing attribute's extension counter is the same sum over the seed
    edges of the proposing set size (out(a1) for the star, out(a2) for the
    fan)."""
    src, dst = rmat22
    n = 1 << 22
    es, ed = distinct_edges(src, dst)
    out = np.bincount(es.astype(np.int64), minlength=n).astype(object)
    inn = np.bincount(ed.astype(np.int64), minlength=n).astype(object)
    c = gj.Context(0)
    c.set_option("factorise", 1)
    G = gj.Graph(c, src, dst, n)
    star = gj.count(c, G, gj.Query(c, *Q.STAR3))
    fan = gj.count(c, G, gj.Query(c, *Q.FAN))
    assert star["matches"] == int(sum(out ** 3))
    assert star["extensions"][2] == star["extensions"][3] == int(sum(out ** 2))
    assert fan["matches"] == int(sum(inn * out ** 2))
    assert fan["extensions"][2] == fan["extensions"][3] == int(sum(inn * out))
    G.close()
    c.close()


def test_rmat22_triangle_index(gj, rmat22):
    """The triangle relation at scale 22 has as many entries as the owner
    kernel counts triangles, and the 4-clique over it counts what the plain
    4-clique counts on sampled seed slices."""
    src, dst = rmat22
    n = 1 << 22
    c = gj.Context(0)
    G = gj.Graph(c, src, dst, n)
    tri = gj.count(c, G, gj.Query(c, *Q.TRIANGLE))["matches"]
    assert G.index_triangles() == tri
    t4 = gj.Query(c, Q.TRI_CLIQUE4[0], Q.TRI_CLIQUE4[1], Q.TRI_CLIQUE4[2], tris=Q.TRI_CLIQUE4[4])
    k4 = gj.Query(c, *Q.CLIQUE4)
    E = G.info()["edges"]
    for lo, hi in slices(E, 6, 20000):
        a, b = gj.count(c, G, t4, lo, hi), gj.count(c, G, k4, lo, hi)
        assert a["matches"] == b["matches"] and a["prefixes"][3] == b["prefixes"][3], (lo, hi)
    G.close()
    c.close()


@pytest.mark.parametrize("name", ["diamond", "cycle4"])
def test_rmat18_2path_counts_agree(gj, name):
    """The diamond and 4-cycle counts by 2-path counts (default) and by the
    generic per-candidate path (strategy 1) agree on counts and every
    counter at R-MAT scale 18."""
    src, dst = synth.rmat_draws(18, seed=0)
    n = 1 << 18
    res = []
    for strategy in (0, 1):
        c = gj.Context(0)
        c.set_option("strategy", strategy)
        G = gj.Graph(c, src, dst, n)
        r = gj.count(c, G, gj.Query(c, *Q.ALL[name]))
        res.append((r["matches"], r["prefixes"], r["extensions"]))
        G.close()
        c.close()
    assert res[0] == res[1]
    assert res[0][0] > 0
