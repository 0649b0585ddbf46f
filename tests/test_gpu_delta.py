"""GPU parity of the delta-query path (gj_apply_updates through the C ABI)
against the CPU oracle's Delta-GJ: signed consolidated rows, count deltas,
raw emissions, per-stage counters, no-op counts and the new edge set."""
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


def _dev(p, n, dtype=np.uint32):
    hip = ctypes.CDLL("libamdhip64.so")
    a = np.empty(n, dtype)
    if n:
        assert hip.hipMemcpy(ctypes.c_void_p(a.ctypes.data), ctypes.c_void_p(p), ctypes.c_size_t(a.nbytes), 2) == 0
    return a


def check_index(G, es, ed):
    """Both directions of the current version (rows, values and row
    pointers) and the largest degrees against the edge list (es, ed), sorted
    by (src, dst)."""
    info = G.info()
    n, E = info["vertices"], info["edges"]
    assert E == len(es)
    order = np.lexsort((es, ed))  # by (dst, src)
    for rev, (rows, cols) in enumerate(((es, ed), (ed[order], es[order]))):
        rp, col, row = G.csr_ptrs(rev)
        assert np.array_equal(_dev(row, E), rows) and np.array_equal(_dev(col, E), cols), rev
        want_rp = np.searchsorted(rows, np.arange(n + 1, dtype=np.uint64)).astype(np.uint32)
        assert np.array_equal(_dev(rp, n + 1), want_rp), rev
    deg_out = np.bincount(es, minlength=n) if E else np.zeros(n, np.int64)
    deg_in = np.bincount(ed, minlength=n) if E else np.zeros(n, np.int64)
    assert (info["max_out"], info["max_in"]) == (int(deg_out.max(initial=0)), int(deg_in.max(initial=0)))


def step(gj, ctx, G, O, qs_py, qs_gj, bs, bd, bg):
    res = gj.apply_updates(ctx, G, bs, bd, bg, qs_gj, rows=True)
    first = True
    O_before = O.copy()
    for q, r in zip(qs_py, res):
        Oq = O_before.copy()
        ref = oracle.delta(Oq, bs, bd, bg, q)
        assert r["count_delta"] == ref["count_delta"], (q, r["count_delta"], ref["count_delta"])
        assert r["n_delta"] == len(ref["rows"])
        assert np.array_equal(r["rows"], ref["rows"]), q
        assert np.array_equal(r["signs"], ref["signs"]), q
        assert r["stats"]["raw_emissions"] == ref["raw_emissions"]
        assert r["stats"]["prefixes"] == ref["prefixes"]
        assert r["stats"]["extensions"] == ref["extensions"]
        if first:
            bi, bd_ = O_before.noops()
            ni, nd = Oq.noops()
            assert (r["stats"]["noop_inserts"], r["stats"]["noop_deletes"]) == (ni - bi, nd - bd_)
            first = False
    oracle.delta(O, bs, bd, bg)  # advance the reference graph
    es, ed = O.edge_list()
    check_index(G, np.asarray(es, np.uint32), np.asarray(ed, np.uint32))
    return res


def test_forced_cancellation(gj, ctx):
    G = gj.Graph(ctx, np.array([2, 1], np.uint32), np.array([3, 3], np.uint32), 4)
    q = gj.Query(ctx, *Q.TRIANGLE)
    r = gj.apply_updates(ctx, G, np.array([1, 2], np.uint32), np.array([2, 3], np.uint32),
                         np.array([1, -1], np.int8), [q], rows=True)[0]
    assert r["stats"]["raw_emissions"] == 2
    assert r["count_delta"] == 0 and r["n_delta"] == 0
    assert G.info()["edges"] == 2 and G.info()["version"] == 1


@pytest.mark.parametrize("names", [("triangle", "cyclic_triangle", "reciprocal"),
                                   ("clique4", "diamond", "cycle4", "paper_diamond")])
def test_random_batches(gj, ctx, names):
    n = 30
    rng = np.random.default_rng(len(names))
    src = rng.integers(0, n, 200).astype(np.uint32)
    dst = rng.integers(0, n, 200).astype(np.uint32)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    qs_py = [Q.ALL[k] for k in names]
    qs_gj = [gj.Query(ctx, *q) for q in qs_py]
    for it in range(8):
        b = int(rng.integers(1, 40))
        bs = rng.integers(0, n, b).astype(np.uint32)
        bd = rng.integers(0, n, b).astype(np.uint32)
        bg = np.where(rng.random(b) < 0.4, -1, 1).astype(np.int8)
        es, ed = O.edge_list()
        for k in range(b):
            if bg[k] < 0 and len(es) and rng.random() < 0.6:
                j = rng.integers(0, len(es))
                bs[k], bd[k] = es[j], ed[j]
        dels = {(int(x), int(y)) for x, y, g in zip(bs, bd, bg) if g < 0}
        keep = np.array([not (g > 0 and (int(x), int(y)) in dels) for x, y, g in zip(bs, bd, bg)])
        step(gj, ctx, G, O, qs_py, qs_gj, bs[keep], bd[keep], bg[keep])


def test_rmat_update_stream(gj, ctx):
    """Base R-MAT scale 11 (seed 0), then a stream of log-uniform batches
    (sizes in [1, 2,000], 10% deletions of base edges, seed 1)."""
    scale = 11
    src, dst = synth.rmat_draws(scale, seed=0)
    n = 1 << scale
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    qs_py = [Q.TRIANGLE, Q.CLIQUE4]
    qs_gj = [gj.Query(ctx, *q) for q in qs_py]
    for k, bs, bd, bg in synth.update_stream(scale, 0, 1, 6, 1, 2000):
        step(gj, ctx, G, O, qs_py, qs_gj, bs, bd, bg)
    # counts of the final graph agree too
    for q, qg in zip(qs_py, qs_gj):
        assert gj.count(ctx, G, qg)["matches"] == oracle.run(O, q)["matches"]


def test_overflow_then_fetch(gj, ctx):
    """A too-small row buffer: the batch is applied, the call reports
    GJ_EOVERFLOW with the row count, and gj_last_delta returns the rows."""
    src, dst = synth.rmat_draws(9, seed=8)
    n = 1 << 9
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    q = gj.Query(ctx, *Q.TRIANGLE)
    (k, bs, bd, bg), = list(synth.update_stream(9, 8, 9, 1, 300, 300))
    ref = oracle.delta(O, bs, bd, bg, Q.TRIANGLE)
    assert len(ref["rows"]) > 3
    r = gj.apply_updates(ctx, G, bs, bd, bg, [q], rows=True, cap=2)[0]
    assert r["n_delta"] == len(ref["rows"])
    assert np.array_equal(r["rows"], ref["rows"]) and np.array_equal(r["signs"], ref["signs"])
    with pytest.raises(gj.GJError) as e:
        gj.last_delta(ctx, 0, 3, 1)
    assert e.value.status == gj.GJ_EOVERFLOW
    rows, signs = gj.last_delta(ctx, 0, 3, len(ref["rows"]))
    assert np.array_equal(rows, ref["rows"])
    with pytest.raises(gj.GJError):
        gj.last_delta(ctx, 1, 3, 10)


def test_count_only_matches_rows(gj, ctx):
    src, dst = synth.rmat_draws(10, seed=5)
    n = 1 << 10
    G1 = gj.Graph(ctx, src, dst, n)
    G2 = gj.Graph(ctx, src, dst, n)
    q = gj.Query(ctx, *Q.TRIANGLE)
    for k, bs, bd, bg in synth.update_stream(10, 5, 7, 4, 1, 500):
        a = gj.apply_updates(ctx, G1, bs, bd, bg, [q], rows=False)[0]
        b = gj.apply_updates(ctx, G2, bs, bd, bg, [q], rows=True)[0]
        assert a["count_delta"] == b["count_delta"] == int(b["signs"].astype(np.int64).sum())


def test_conflict_and_bad_input(gj, ctx):
    G = gj.Graph(ctx, np.array([0, 1], np.uint32), np.array([1, 2], np.uint32), 5)
    q = gj.Query(ctx, *Q.TRIANGLE)
    with pytest.raises(gj.GJError) as e:
        gj.apply_updates(ctx, G, np.array([3, 3], np.uint32), np.array([4, 4], np.uint32),
                         np.array([1, -1], np.int8), [q])
    assert e.value.status == gj.GJ_EINVAL
    with pytest.raises(gj.GJError) as e:
        gj.apply_updates(ctx, G, np.array([7], np.uint32), np.array([1], np.uint32),
                         np.array([1], np.int8), [q])
    assert e.value.status == gj.GJ_EINVAL
    with pytest.raises(gj.GJError) as e:
        gj.apply_updates(ctx, G, np.array([2], np.uint32), np.array([1], np.uint32),
                         np.array([3], np.int8), [q])
    assert e.value.status == gj.GJ_EINVAL
    assert G.info()["edges"] == 2 and G.info()["version"] == 0
    # empty and all-no-op batches leave the version unchanged
    r = gj.apply_updates(ctx, G, np.array([0, 4], np.uint32), np.array([1, 4], np.uint32),
                         np.array([1, 1], np.int8), [q])[0]
    assert r["count_delta"] == 0 and r["stats"]["noop_inserts"] == 1
    assert G.info()["version"] == 0


def test_fused_delta_equals_depth_first(gj):
    """Count-only deltas through the fused pipeline (one launch for every dQ_i
    of every query) equal the depth-first path and the oracle."""
    scale = 11
    src, dst = synth.rmat_draws(scale, seed=12)
    n = 1 << scale
    cf = gj.Context(0)
    cp = gj.Context(0)
    cp.set_option("delta_fused", 0)
    Gf, Gp = gj.Graph(cf, src, dst, n), gj.Graph(cp, src, dst, n)
    names = ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4", "reciprocal"]
    qf = [gj.Query(cf, *Q.ALL[k]) for k in names]
    qp = [gj.Query(cp, *Q.ALL[k]) for k in names]
    O = oracle.Graph(n, src, dst)
    for k, bs, bd, bg in synth.update_stream(scale, 12, 13, 5, 1, 3000):
        rf = gj.apply_updates(cf, Gf, bs, bd, bg, qf)
        rp = gj.apply_updates(cp, Gp, bs, bd, bg, qp)
        for name, a, b in zip(names, rf, rp):
            ref = oracle.delta(O.copy(), bs, bd, bg, Q.ALL[name])
            assert a["count_delta"] == b["count_delta"] == ref["count_delta"], name
            for key in ("raw_emissions", "prefixes", "extensions", "noop_inserts", "noop_deletes"):
                assert a["stats"][key] == b["stats"][key] == (ref[key] if key in ref else b["stats"][key]), key
        oracle.delta(O, bs, bd, bg)
    assert cf.get_option("batch_fallbacks") == 0


def test_owner_delta_equals_depth_first(gj):
    """Count-only deltas of the triangle shapes through the owner-grouped
    kernel (forced for every batch size) equal the depth-first path and the
    oracle, counters included; other queries in the same call take the fused
    pipeline."""
    scale = 11
    src, dst = synth.rmat_draws(scale, seed=14)
    n = 1 << scale
    co = gj.Context(0)
    co.set_option("delta_owner_min", 1)
    assert co.get_option("delta_owner_min") == 1
    cp = gj.Context(0)
    cp.set_option("delta_fused", 0)
    Go, Gp = gj.Graph(co, src, dst, n), gj.Graph(cp, src, dst, n)
    names = ["triangle", "cyclic_triangle", "diamond", "clique4"]
    qo = [gj.Query(co, *Q.ALL[k]) for k in names]
    qp = [gj.Query(cp, *Q.ALL[k]) for k in names]
    O = oracle.Graph(n, src, dst)
    for k, bs, bd, bg in synth.update_stream(scale, 14, 15, 6, 1, 4000):
        ro = gj.apply_updates(co, Go, bs, bd, bg, qo)
        rp = gj.apply_updates(cp, Gp, bs, bd, bg, qp)
        for name, a, b in zip(names, ro, rp):
            ref = oracle.delta(O.copy(), bs, bd, bg, Q.ALL[name])
            assert a["count_delta"] == b["count_delta"] == ref["count_delta"], name
            for key in ("raw_emissions", "prefixes", "extensions", "noop_inserts", "noop_deletes"):
                assert a["stats"][key] == b["stats"][key], (name, key)
            if name in ("triangle", "cyclic_triangle") and a["stats"]["raw_emissions"]:
                assert a["stats"]["kernel_launches"] == 3  # one owner launch per dQ_i
        oracle.delta(O, bs, bd, bg)
    with pytest.raises(gj.GJError):
        co.set_option("delta_owner_min", -1)
