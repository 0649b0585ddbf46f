"""GPU parity of the last-stage counts grouped by prefix runs (run.hip)
against the CPU oracle: counts and per-stage counters of every test query in
several orders, with and without inequalities, membership tables, many
tasks per run and both sides of the size-ratio switch; signed counts of the
depth-first delta queries; and runs whose shared set is too large for LDS
next to staged ones in one stage."""
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


def run_ctx(gj, task_work=1 << 15, ratio=8, min_work=0, hash_index=1):
    c = gj.Context(0)
    c.set_option("run_stage_min", 0)  # every last stage that can, however small
    c.set_option("run_min_tasks", 0)  # and however few tasks it makes
    c.set_option("run_min_work", min_work)
    c.set_option("run_task_work", task_work)
    c.set_option("run_ratio", ratio)
    c.set_option("hash_index", hash_index)
    c.set_option("hash_build_work", 0)
    return c


def check(gj, c, G, O, q, seed_lo=0, seed_hi=None):
    """Counts and counters over [seed_lo, seed_hi); the whole edge range is
    taken as two slices, so that the whole-count kernels (owner-grouped,
    edge-grouped, 2-path) stay out and every stage runs on the depth-first
    path."""
    E = G.info()["edges"]
    hi = E if seed_hi is None else min(seed_hi, E)
    cuts = [seed_lo, hi] if (seed_lo, hi) != (0, E) else [0, E // 2, E]
    Qh = gj.Query(c, *q)
    for lo_, hi_ in zip(cuts[:-1], cuts[1:]):
        ref = oracle.run(O, q, seed_lo=lo_, seed_hi=hi_, threads=8)
        got = gj.count(c, G, Qh, lo_, hi_)
        assert got["matches"] == ref["matches"], (q, lo_, hi_, got["matches"], ref["matches"])
        assert got["prefixes"] == ref["prefixes"], q
        assert got["extensions"] == ref["extensions"], q
    return ref


# (task_work, ratio): runs cut into as many tasks as they have prefixes, or
# kept whole; new sets always streamed, never streamed, or by the default ratio
SETTINGS = [(1, 8), (64, 0), (1 << 15, 64), (1 << 15, 8)]


@pytest.mark.parametrize("name", sorted(Q.ALL))
@pytest.mark.parametrize("task_work,ratio", SETTINGS)
def test_queries_all_orders(gj, name, task_work, ratio):
    q = Q.ALL[name]
    c = run_ctx(gj, task_work, ratio)
    scale = 10 if q[0] <= 4 else 8
    src, dst = synth.rmat_draws(scale, seed=11)
    n = 1 << scale
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    orders = Q.valid_orders(q)
    before = c.get_option("run_tasks")
    for order in orders[:: max(1, len(orders) // 4)]:
        check(gj, c, G, O, Q.with_order(q, order))
    assert c.get_option("run_tasks") > before, name  # the run kernels took part


@pytest.mark.parametrize("name", ["triangle", "clique4", "diamond", "cycle4", "house", "clique5"])
def test_inequalities_and_symmetric(gj, name):
    """Random inequality sets (several orders) on a directed R-MAT graph, and
    the symmetry-breaking sets on its undirected form."""
    rng = np.random.default_rng(len(name) + 100)
    c = run_ctx(gj, task_work=256)
    scale = 10 if Q.ALL[name][0] <= 4 else 8
    src, dst = synth.rmat_draws(scale, seed=12)
    n = 1 << scale
    q = Q.ALL[name]
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    orders = Q.valid_orders(q)
    for order in [orders[0], orders[len(orders) // 2], orders[-1]]:
        m = q[0]
        less = []
        for _ in range(int(rng.integers(1, m))):
            x, y = rng.choice(m, 2, replace=False)
            if (int(y), int(x)) not in less:
                less.append((int(x), int(y)))
        check(gj, c, G, O, Q.with_less(Q.with_order(q, order), less))
    if name in Q.SYM_LESS:
        u, v = oracle.symmetric_edges(n, src, dst)
        Gu, Ou = gj.Graph(c, src, dst, n, undirected=True), oracle.Graph(n, u, v)
        check(gj, c, Gu, Ou, Q.with_less(q, Q.SYM_LESS[name][0]))


@pytest.mark.parametrize("hash_index", [0, 1])
def test_seed_slices_rmat(gj, hash_index):
    """Seed slices of an R-MAT-14 graph, hub rows included, at the default
    run sizes and split (stage and task-count thresholds lowered so that the
    run kernels take part at this scale)."""
    c = gj.Context(0)
    c.set_option("hash_index", hash_index)
    c.set_option("hash_build_work", 0)
    c.set_option("run_min_tasks", 0)
    c.set_option("run_stage_min", 0)
    src, dst = synth.rmat_draws(14, seed=13)
    n = 1 << 14
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    E = G.info()["edges"]
    before = c.get_option("run_tasks")
    for q in (Q.CLIQUE4, Q.DIAMOND, Q.CYCLE4, Q.TRIANGLE):
        for lo in (0, E // 3, E - 4000):
            check(gj, c, G, O, q, lo, lo + 4000)
    assert c.get_option("run_tasks") > before


def test_large_shared_sets_next_to_small(gj):
    """One stage with runs whose shared set exceeds the LDS table (hubs with
    6,000, 4,200 and 4,097 out-neighbours, all pairwise linked) beside runs
    that are staged: the large ones go to the per-candidate kernel, and the
    total is exact."""
    rng = np.random.default_rng(14)
    n = 12000
    hubs = [0, 1, 2]
    src, dst = [], []
    for h, k in zip(hubs, (6000, 4200, 4097)):
        nb = rng.choice(np.arange(3, n), k, replace=False)
        src += [h] * k
        dst += list(nb)
    for h in hubs:
        for g in hubs:
            if h != g:
                src.append(h)
                dst.append(g)
    s2, d2 = synth.rmat_draws(13, seed=14)
    src = np.concatenate([np.array(src, np.uint32), s2 % n]).astype(np.uint32)
    dst = np.concatenate([np.array(dst, np.uint32), d2 % n]).astype(np.uint32)
    c = run_ctx(gj, task_work=4096)
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    big0 = c.get_option("run_tasks_big")
    for q in (Q.TRIANGLE, Q.CLIQUE4, Q.DIAMOND, Q.CYCLE4):
        check(gj, c, G, O, q)
    assert c.get_option("run_tasks_big") > big0  # the large-set shape took the hub runs


def test_sets_beyond_both_tables(gj):
    """Shared sets of 25,001 and 26,000 values (above the large shape's
    24,576): those runs go to the per-candidate kernel, next to staged runs
    of both shapes.  The hubs are the last two vertices, so seed ranges that
    stop before their rows keep the oracle's diamond work small."""
    rng = np.random.default_rng(18)
    n = 40000
    h, h2 = n - 1, n - 2
    s0, d0 = synth.rmat_draws(12, seed=18)
    src = [s0 % (n - 2)]
    dst = [d0 % (n - 2)]
    src.append(np.full(26000, h)); dst.append(rng.choice(n - 2, 26000, replace=False))
    src.append(rng.choice(n - 2, 400, replace=False)); dst.append(np.full(400, h))
    src.append(np.full(25000, h2)); dst.append(rng.choice(n - 2, 25000, replace=False))
    src.append(np.array([h2])); dst.append(np.array([h]))
    src = np.concatenate(src).astype(np.uint32)
    dst = np.concatenate(dst).astype(np.uint32)
    c = run_ctx(gj, task_work=1 << 14)
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    E = G.info()["edges"]
    end_h = E - 26000  # first edge of h's row
    end_h2 = end_h - 25001  # first edge of h2's row
    w0 = c.get_option("run_w_large")
    for q in (Q.TRIANGLE, Q.DIAMOND, Q.CYCLE4):
        check(gj, c, G, O, q, 0, end_h2)
    check(gj, c, G, O, Q.CLIQUE4, 0, end_h)
    assert c.get_option("run_w_large") > w0  # some runs exceeded both shapes


@pytest.mark.parametrize("task_work", [1, 1 << 15])
def test_delta_depth_first(gj, task_work):
    """Delta queries on the depth-first path (signed weights carried by the
    prefixes) keep the per-candidate kernel beside static counts that take
    the run kernels on the same context: count deltas equal the oracle's
    Delta-GJ batch by batch."""
    c = run_ctx(gj, task_work=task_work)
    c.set_option("delta_fused", 0)
    scale = 10
    src, dst = synth.rmat_draws(scale, seed=15)
    n = 1 << scale
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    qs = [Q.TRIANGLE, Q.CLIQUE4, Q.DIAMOND, Q.CYCLE4, Q.HOUSE]
    hs = [gj.Query(c, *q) for q in qs]
    for k, bs, bd, bg in synth.update_stream(scale, 15, 16, 5, 1, 3000):
        before = c.get_option("run_tasks")
        res = gj.apply_updates(c, G, bs, bd, bg, hs, rows=False)
        assert c.get_option("run_tasks") == before
        for q, r in zip(qs, res):
            ref = oracle.delta(O.copy(), bs, bd, bg, q, rows=False, threads=8)
            assert r["count_delta"] == ref["count_delta"], (k, q, r["count_delta"], ref["count_delta"])
            assert r["stats"]["prefixes"] == ref["prefixes"] and r["stats"]["extensions"] == ref["extensions"]
        oracle.delta(O, bs, bd, bg)
        E = G.info()["edges"]
        check(gj, c, G, O, Q.CLIQUE4, 0, E // 2)


def test_off_equals_on(gj):
    """run_stage 0 and 1 give the same counts and counters on an R-MAT-12
    graph for every test query."""
    src, dst = synth.rmat_draws(12, seed=17)
    n = 1 << 12
    on = run_ctx(gj)
    off = gj.Context(0)
    off.set_option("run_stage", 0)
    Gon, Goff = gj.Graph(on, src, dst, n), gj.Graph(off, src, dst, n)
    for name in ("triangle", "cyclic_triangle", "clique4", "diamond", "paper_diamond", "cycle4", "reciprocal"):
        q = Q.ALL[name]
        E = Gon.info()["edges"]
        a = gj.count(on, Gon, gj.Query(on, *q), 1, E)
        b = gj.count(off, Goff, gj.Query(off, *q), 1, E)
        assert (a["matches"], a["prefixes"], a["extensions"]) == (b["matches"], b["prefixes"], b["extensions"]), name


def test_declined_stages(gj):
    """A stage whose staged runs make fewer tasks than run_min_tasks is left
    whole to the per-candidate kernel: counts and counters still equal the
    oracle's, and the context counts the declined stages."""
    c = run_ctx(gj)
    c.set_option("run_min_tasks", 1 << 40)
    src, dst = synth.rmat_draws(11, seed=19)
    n = 1 << 11
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    for q in (Q.TRIANGLE, Q.CLIQUE4, Q.DIAMOND):
        check(gj, c, G, O, q)
    assert c.get_option("run_declined") > 0 and c.get_option("run_tasks") == 0


def batch_requests(gj, c, E, rng, nreq, names, widths):
    qs = {k: gj.Query(c, *Q.ALL[k]) for k in names}
    reqs, specs = [], []
    for i in range(nreq):
        k = names[i % len(names)]
        lo = 0 if i < len(names) else int(rng.integers(0, E))  # the first of each query at the hub rows
        w = int(rng.choice(widths))
        reqs.append((qs[k], lo, min(lo + w, E)))
        specs.append((Q.ALL[k], lo, min(lo + w, E)))
    return reqs, specs


@pytest.mark.parametrize("task_work,ratio", [(1, 8), (1 << 15, 2), (64, 0)])
def test_batched_pipeline_runs(gj, task_work, ratio):
    """The fused pipeline's last stages grouped by runs (batch_run): every
    request's count and counters equal the oracle's over three replays of
    the captured pipeline with different request mixes (queries ending at
    different levels share them), and the run kernels took part."""
    c = run_ctx(gj, task_work, ratio)
    c.set_option("run_reuse", 1)
    c.set_option("batch_heavy", 0)  # every request fused
    assert c.get_option("batch_run") == 1
    src, dst = synth.rmat_draws(12, seed=31)
    n = 1 << 12
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    E = O.num_edges
    rng = np.random.default_rng(task_work + ratio)
    names = ["clique4", "diamond", "triangle", "cycle4", "paper_diamond", "cyclic_triangle", "house"]
    b0 = c.get_option("run_builds")
    for rep in range(3):
        reqs, specs = batch_requests(gj, c, E, rng, 24 + 5 * rep, names[rep:] + names[:rep], [0, 1, 40, 400, 2500])
        counts, stats = gj.run_batch(c, G, reqs)
        assert c.get_option("batch_fallbacks") == 0
        for (q, lo, hi), cnt, st in zip(specs, counts, stats):
            ref = oracle.run(O, q, seed_lo=lo, seed_hi=hi, threads=8)
            assert (cnt, st["prefixes"], st["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"]), \
                (rep, q, lo, hi)
    assert c.get_option("run_builds") > b0


def test_batched_runs_off_equals_on(gj):
    """batch_run 0 and 1 give the same counts and counters at the default
    run sizes, with inequalities on the symmetric graph among the requests;
    switching the option re-captures the pipeline."""
    src, dst = synth.rmat_draws(13, seed=32)
    n = 1 << 13
    c = gj.Context(0)
    c.set_option("batch_heavy", 0)
    G = gj.Graph(c, src, dst, n)
    Gu = gj.Graph(c, src, dst, n, undirected=True)
    E = G.info()["edges"]
    rng = np.random.default_rng(33)
    reqs, _ = batch_requests(gj, c, E, rng, 30, ["clique4", "diamond", "triangle", "cycle4"], [100, 3000])
    qs = [gj.Query(c, *Q.with_less(Q.ALL[k], Q.SYM_LESS[k][0])) for k in ("clique4", "triangle")]
    Eu = Gu.info()["edges"]
    ureqs = [(qs[i % 2], lo, lo + 3000) for i, lo in enumerate(range(0, Eu, Eu // 6))]
    def key(out):
        counts, stats = out
        return counts, [(s["matches"], s["prefixes"], s["extensions"]) for s in stats]

    res = {}
    for on in (1, 0, 1):
        c.set_option("batch_run", on)
        a = key(gj.run_batch(c, G, reqs))
        b = key(gj.run_batch(c, Gu, ureqs))
        if on in res:
            assert res[on] == (a, b)
        res[on] = (a, b)
    assert res[0] == res[1]
    assert sum(res[1][0][0]) > 0 and sum(res[1][1][0]) > 0


def test_small_shape_only(gj):
    """run_big 0 (the server's light lane): runs whose shared set needs the
    large shape stay with the per-candidate kernel, the rest are staged in
    the small shape; counts and counters equal the oracle's on the depth-first
    path and in the fused pipeline, and the large shape takes no task."""
    rng = np.random.default_rng(21)
    n = 9000
    src, dst = [], []
    for h, k in ((0, 5000), (1, 4500)):
        nb = rng.choice(np.arange(2, n), k, replace=False)
        src += [h] * k
        dst += list(nb)
    src += [0, 1]
    dst += [1, 0]
    s2, d2 = synth.rmat_draws(12, seed=22)
    src = np.concatenate([np.array(src, np.uint32), s2 % n]).astype(np.uint32)
    dst = np.concatenate([np.array(dst, np.uint32), d2 % n]).astype(np.uint32)
    c = run_ctx(gj, task_work=4096)
    c.set_option("run_big", 0)
    assert c.get_option("run_big") == 0
    c.set_option("batch_heavy", 0)
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    big0, t0 = c.get_option("run_tasks_big"), c.get_option("run_tasks")
    for q in (Q.TRIANGLE, Q.CLIQUE4, Q.DIAMOND):
        check(gj, c, G, O, q)
    assert c.get_option("run_tasks") > t0 and c.get_option("run_tasks_big") == big0
    E = O.num_edges
    qs = {k: gj.Query(c, *Q.ALL[k]) for k in ("clique4", "diamond", "triangle")}
    reqs = [(qs[k], lo, min(E, lo + 3000)) for k in qs for lo in (0, E // 2)]
    counts, stats = gj.run_batch(c, G, reqs)
    for (qh, lo, hi), (k, _), cnt, st in zip(reqs, [(k, 0) for k in qs for _ in (0, 1)], counts, stats):
        ref = oracle.run(O, Q.ALL[k], seed_lo=lo, seed_hi=hi, threads=8)
        assert (cnt, st["prefixes"], st["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"]), (k, lo)
    with pytest.raises(gj.GJError):
        c.set_option("run_big", 2)
