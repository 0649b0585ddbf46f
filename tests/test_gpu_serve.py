"""Served form: requests submitted to the server (continuously batched, in
one mix with update batches, from several threads) return exactly what the
same requests return issued alone, in submission order, on a separate
replica of the graph."""
import threading

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


def make_requests(rng, E, n_counts, names):
    out = []
    for i in range(n_counts):
        lo = int(rng.integers(0, E))
        out.append((names[i % len(names)], lo, lo + int(rng.integers(0, 400))))
    return out


def replay_and_check(gj, src, dst, n, submitted, results):
    """submitted: [(ticket, ("count", name, lo, hi) | ("update", bs, bd, bg, names))] in ticket order."""
    ref_ctx = gj.Context(0)
    ref_ctx.set_option("delta_fused", 0)
    G = gj.Graph(ref_ctx, src, dst, n)
    qs = {k: gj.Query(ref_ctx, *Q.ALL[k]) for k in Q.ALL}
    version = 0
    O = oracle.Graph(n, src, dst)
    for ticket, req in sorted(submitted, key=lambda x: x[0]):
        r = results[ticket]
        assert r["status"] == 0
        if req[0] == "count":
            _, name, lo, hi = req
            alone = gj.count(ref_ctx, G, qs[name], lo, hi)["matches"]
            assert r["count"] == alone, (ticket, name, lo, hi)
            assert r["count"] == oracle.run(O, Q.ALL[name], seed_lo=lo, seed_hi=hi)["matches"]
            assert r["version"] == version
        else:
            _, bs, bd, bg, names = req
            alone = gj.apply_updates(ref_ctx, G, bs, bd, bg, [qs[k] for k in names])
            version = G.info()["version"]
            assert r["count_delta"] == [a["count_delta"] for a in alone]
            assert r["version"] == version
            oracle.delta(O, bs, bd, bg)


@pytest.mark.parametrize("iteration_work,versions,heavy_work", [(None, None, None), (0, 2, None), (4096, 3, 2048),
                                                                (1 << 16, 8, None), (256, 4, 1 << 14)])
def test_served_mix_equals_alone(gj, iteration_work, versions, heavy_work):
    """iteration_work 0: whole requests in arrival order; small budgets: most
    requests heavy, cut into many chunks on the heavy lanes; versions:
    resident version slots."""
    scale = 11
    src, dst = synth.rmat_draws(scale, seed=31)
    n = 1 << scale
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    qs = {k: gj.Query(ctx, *Q.ALL[k]) for k in Q.ALL}
    E = G.info()["edges"]
    rng = np.random.default_rng(5)
    srv = gj.Server(ctx, G, max_batch=32, iteration_work=iteration_work, versions=versions)
    if heavy_work is not None:
        srv.set_option("heavy_work", heavy_work)
    submitted = []
    stream = list(synth.update_stream(scale, 31, 32, 6, 1, 500))
    names = ["triangle", "clique4", "diamond", "cycle4", "cyclic_triangle", "reciprocal"]
    for k in range(6):
        for name, lo, hi in make_requests(rng, E, 25, names):
            submitted.append((srv.submit_count(qs[name], lo, hi), ("count", name, lo, hi)))
        _, bs, bd, bg = stream[k]
        upd_names = ["triangle", "clique4", "diamond"]
        submitted.append((srv.submit_update(bs, bd, bg, [qs[x] for x in upd_names]),
                          ("update", bs, bd, bg, upd_names)))
    results = {t: srv.wait(t) for t, _ in submitted}
    st = srv.stats()
    srv.close()
    assert st["completed_counts"] == 150 and st["completed_updates"] == 6
    if iteration_work != 256:  # 256: nearly every request is heavy
        assert max(r["batch_size"] for r in results.values()) > 1  # requests were batched
    if iteration_work == 4096:
        assert st["count_batches"] > 150  # requests were cut into chunks
    replay_and_check(gj, src, dst, n, submitted, results)


def test_served_from_threads(gj):
    scale = 10
    src, dst = synth.rmat_draws(scale, seed=41)
    n = 1 << scale
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    qs = {k: gj.Query(ctx, *Q.ALL[k]) for k in Q.ALL}
    E = G.info()["edges"]
    srv = gj.Server(ctx, G, max_batch=16, mem_budget_bytes=1 << 24)
    submitted, lock = [], threading.Lock()
    stream = list(synth.update_stream(scale, 41, 42, 4, 1, 300))

    def client(cid):
        rng = np.random.default_rng(100 + cid)
        for name, lo, hi in make_requests(rng, E, 30, ["triangle", "clique4", "cycle4"]):
            t = srv.submit_count(qs[name], lo, hi)
            with lock:
                submitted.append((t, ("count", name, lo, hi)))
            if cid == 0 and rng.random() < 0.15 and stream:
                _, bs, bd, bg = stream.pop()
                with lock:
                    t = srv.submit_update(bs, bd, bg, [qs["triangle"]])
                    submitted.append((t, ("update", bs, bd, bg, ["triangle"])))

    threads = [threading.Thread(target=client, args=(i,)) for i in range(4)]
    for th in threads:
        th.start()
    for th in threads:
        th.join()
    results = {t: srv.wait(t, 60000) for t, _ in submitted}
    srv.close()
    replay_and_check(gj, src, dst, n, submitted, results)


def test_served_versions_with_noop_and_rejected_updates(gj):
    """Counts interleaved with many small updates submitted at once (the
    update thread runs ahead of the counts it must not overwrite), an update
    made only of no-ops (the version does not change) and a rejected one
    (vertex out of range: an error status, the graph unchanged)."""
    scale = 10
    src, dst = synth.rmat_draws(scale, seed=51)
    n = 1 << scale
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    qs = {k: gj.Query(ctx, *Q.ALL[k]) for k in Q.ALL}
    E = G.info()["edges"]
    srv = gj.Server(ctx, G, max_batch=8, iteration_work=1 << 14, versions=3)
    stream = list(synth.update_stream(scale, 51, 52, 10, 1, 200))
    rng = np.random.default_rng(9)
    submitted, rejected = [], None
    for k in range(12):
        for name, lo, hi in make_requests(rng, E, 3, ["triangle", "clique4"]):
            submitted.append((srv.submit_count(qs[name], lo, hi), ("count", name, lo, hi)))
        # a full-range count too (the owner-grouped kernel when it runs alone)
        submitted.append((srv.submit_count(qs["triangle"]), ("count", "triangle", 0, 1 << 40)))
        if k == 4:
            # re-insert edges already present: all no-ops
            bs, bd = np.asarray(src[:50], np.uint32), np.asarray(dst[:50], np.uint32)
            keep = bs != bd
            bs, bd = bs[keep], bd[keep]
            bg = np.ones(len(bs), np.int8)
            submitted.append((srv.submit_update(bs, bd, bg, [qs["triangle"]]), ("update", bs, bd, bg, ["triangle"])))
        elif k == 7:
            bs = np.array([1, n + 5], np.uint32)
            bd = np.array([2, 3], np.uint32)
            bg = np.ones(2, np.int8)
            rejected = srv.submit_update(bs, bd, bg, [qs["triangle"]])
        else:
            _, bs, bd, bg = stream.pop(0)
            submitted.append((srv.submit_update(bs, bd, bg, [qs["triangle"], qs["clique4"]]),
                              ("update", bs, bd, bg, ["triangle", "clique4"])))
    results = {t: srv.wait(t, 60000) for t, _ in submitted}
    rej = srv.wait(rejected, 60000)
    srv.close()
    assert rej["status"] != 0 and rej["kind"] == gj.REQ_UPDATE
    noop = [results[t] for t, r in submitted if r[0] == "update" and len(r[4]) == 1][0]
    assert noop["count_delta"] == [0]
    replay_and_check(gj, src, dst, n, submitted, results)


def test_server_options(gj):
    ctx = gj.Context(0)
    src, dst = synth.rmat_draws(8, seed=3)
    G = gj.Graph(ctx, src, dst, 1 << 8)
    q = gj.Query(ctx, *Q.TRIANGLE)
    srv = gj.Server(ctx, G)
    for key, val in (("versions", 1), ("versions", 9), ("iteration_work", -1), ("max_batch", 0), ("nope", 1),
                     ("heavy_lanes", 0), ("heavy_lanes", 5), ("heavy_work", -1), ("update_priority", 2)):
        with pytest.raises(gj.GJError) as e:
            srv.set_option(key, val)
        assert e.value.status == gj.GJ_EINVAL
    srv.set_option("versions", 5)
    srv.set_option("heavy_lanes", 1)
    srv.set_option("update_priority", 0)
    srv.set_option("heavy_work", 1 << 20)
    r = srv.wait(srv.submit_count(q))
    assert r["count"] == oracle.run(oracle.Graph(1 << 8, src, dst), Q.TRIANGLE)["matches"]
    for key in ("versions", "heavy_lanes"):
        with pytest.raises(gj.GJError) as e:
            srv.set_option(key, 3)  # after the first request
        assert e.value.status == gj.GJ_EBUSY
    srv.set_option("iteration_work", 0)
    assert srv.wait(srv.submit_count(q))["count"] == r["count"]
    srv.close()
    G.close()
    ctx.close()


@pytest.mark.parametrize("lanes", [0, 1, 2, 4])
def test_served_update_lanes(gj, lanes):
    """Update batches whose count-only delta queries run side by side on the
    server's delta lanes (delta_lane_min 0: every batch with a change),
    between counts: every count delta equals the same batch applied alone,
    and the oracle's, batch by batch."""
    scale = 11
    src, dst = synth.rmat_draws(scale, seed=51)
    n = 1 << scale
    ctx = gj.Context(0)
    ctx.set_option("delta_lane_min", 0)
    G = gj.Graph(ctx, src, dst, n)
    qs = {k: gj.Query(ctx, *Q.ALL[k]) for k in Q.ALL}
    E = G.info()["edges"]
    srv = gj.Server(ctx, G, max_batch=16)
    srv.set_option("update_lanes", lanes)
    rng = np.random.default_rng(52)
    submitted = []
    upd_names = ["triangle", "clique4", "diamond", "cycle4", "house"]
    for k, bs, bd, bg in synth.update_stream(scale, 51, 53, 5, 1, 2000):
        for name, lo, hi in make_requests(rng, E, 6, ["triangle", "clique4", "diamond"]):
            submitted.append((srv.submit_count(qs[name], lo, hi), ("count", name, lo, hi)))
        submitted.append((srv.submit_update(bs, bd, bg, [qs[x] for x in upd_names]),
                          ("update", bs, bd, bg, upd_names)))
    results = {t: srv.wait(t, 120000) for t, _ in submitted}
    srv.close()
    replay_and_check(gj, src, dst, n, submitted, results)
    O = oracle.Graph(n, src, dst)
    for t, req in sorted(submitted, key=lambda x: x[0]):
        if req[0] != "update":
            continue
        _, bs, bd, bg, names = req
        want = [oracle.delta(O.copy(), bs, bd, bg, Q.ALL[x], rows=False, threads=8)["count_delta"] for x in names]
        assert results[t]["count_delta"] == want, t
        oracle.delta(O, bs, bd, bg)
