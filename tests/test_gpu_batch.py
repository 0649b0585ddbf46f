"""Batched execution (gj_run_batch: fused levels, device-resident sizes,
hipGraph replay) and its autotuner: every request's count and counters equal
the one-at-a-time path and the oracle."""
import os

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


def mixed_requests(gj, ctx, E, rng, nreq):
    names = ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4", "reciprocal", "house",
             "paper_diamond"]
    qs = {k: gj.Query(ctx, *Q.ALL[k]) for k in names}
    qs["edge"] = gj.Query(ctx, 2, [(0, 1)], [1, 0])
    keys = list(qs)
    reqs, specs = [], []
    for i in range(nreq):
        k = keys[i % len(keys)]
        lo = int(rng.integers(0, E))
        width = int(rng.choice([0, 1, 7, 50, 300]))
        reqs.append((qs[k], lo, lo + width))
        specs.append((Q.ALL.get(k, (2, [(0, 1)], [1, 0])), lo, lo + width))
    return reqs, specs


def test_batch_equals_plain_and_oracle(gj):
    src, dst = synth.rmat_draws(11, seed=21)
    n = 1 << 11
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    E = O.num_edges
    rng = np.random.default_rng(1)
    reqs, specs = mixed_requests(gj, ctx, E, rng, 45)
    counts, stats = gj.run_batch(ctx, G, reqs)
    assert ctx.get_option("batch_fallbacks") == 0
    for (qh, lo, hi), (q, _, _), c, st in zip(reqs, specs, counts, stats):
        plain = gj.count(ctx, G, qh, lo, hi)
        ref = oracle.run(O, q, seed_lo=lo, seed_hi=hi)
        assert c == plain["matches"] == ref["matches"], (q, lo, hi)
        assert st["prefixes"] == plain["prefixes"] == ref["prefixes"]
        assert st["extensions"] == plain["extensions"] == ref["extensions"]


def test_replays_with_eager_work_between(gj):
    """The captured pipeline is replayed for different request sets of the
    same shape, with eager library calls and synchronisations in between;
    every replay matches the eager results."""
    src, dst = synth.rmat_draws(12, seed=5)
    n = 1 << 12
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    E = G.info()["edges"]
    rng = np.random.default_rng(2)
    for it in range(5):
        reqs, _ = mixed_requests(gj, ctx, E, rng, 20)
        counts, _ = gj.run_batch(ctx, G, reqs)
        eager = [gj.count(ctx, G, q, lo, hi)["matches"] for q, lo, hi in reqs]
        assert counts == eager, it
    # a larger batch (new capture), then the small shape again
    reqs, _ = mixed_requests(gj, ctx, E, rng, 150)
    counts, _ = gj.run_batch(ctx, G, reqs)
    assert counts == [gj.count(ctx, G, q, lo, hi)["matches"] for q, lo, hi in reqs]


def test_overflow_falls_back(gj):
    src, dst = synth.rmat_draws(10, seed=3)
    n = 1 << 10
    ctx = gj.Context(0)
    ctx.set_option("batch_cap", 64)
    G = gj.Graph(ctx, src, dst, n)
    E = G.info()["edges"]
    q = gj.Query(ctx, *Q.CLIQUE4)
    reqs = [(q, 0, E), (q, 5, 400)]
    counts, stats = gj.run_batch(ctx, G, reqs)
    O = oracle.Graph(n, src, dst)
    assert counts == [oracle.run(O, Q.CLIQUE4)["matches"],
                      oracle.run(O, Q.CLIQUE4, seed_lo=5, seed_hi=400)["matches"]]
    assert ctx.get_option("batch_fallbacks") == 1


def test_batch_after_updates(gj):
    src, dst = synth.rmat_draws(10, seed=4)
    n = 1 << 10
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    q = gj.Query(ctx, *Q.TRIANGLE)
    for k, bs, bd, bg in synth.update_stream(10, 4, 5, 3, 10, 300):
        gj.apply_updates(ctx, G, bs, bd, bg, [q])
        oracle.delta(O, bs, bd, bg)
        E = G.info()["edges"]
        counts, _ = gj.run_batch(ctx, G, [(q, 0, E), (q, 100, 200)])
        assert counts == [oracle.run(O, Q.TRIANGLE)["matches"],
                          oracle.run(O, Q.TRIANGLE, seed_lo=100, seed_hi=200)["matches"]]


def test_autotune_and_cache(gj, tmp_path):
    src, dst = synth.rmat_draws(12, seed=6)
    n = 1 << 12
    ctx = gj.Context(0)
    G = gj.Graph(ctx, src, dst, n)
    E = G.info()["edges"]
    rng = np.random.default_rng(3)
    reqs, _ = mixed_requests(gj, ctx, E, rng, 16)
    path = str(tmp_path / "tune.json")
    t = gj.autotune(ctx, G, reqs, path)
    # the starting point, then each parameter's other values (coordinate descent)
    assert 1 + 1 + 3 + 2 + 2 + 3 + 2 + 1 + 2 <= t["configs_tried"] <= 1 + 2 + 4 + 3 + 3 + 4 + 3 + 2 + 3 \
        and not t["from_cache"]
    assert os.path.exists(path)
    keys = ("batch_lin", "batch_waves_per_cu", "batch_claim_words", "hash_index", "propose_u", "batch_heavy",
            "batch_run", "run_ratio")
    opts = {k: ctx.get_option(k) for k in keys}
    assert opts == {k: t[k] for k in keys}  # the context keeps the choice
    counts, _ = gj.run_batch(ctx, G, reqs)
    assert counts == [gj.count(ctx, G, q, lo, hi)["matches"] for q, lo, hi in reqs]
    ctx2 = gj.Context(0)
    G2 = gj.Graph(ctx2, src, dst, n)
    reqs2 = [(gj.Query(ctx2, q.num_attrs, q.atoms, q.order), lo, hi) for q, lo, hi in reqs]
    t2 = gj.autotune(ctx2, G2, reqs2, path)
    assert t2["from_cache"] and all(t2[k] == t[k] for k in keys)
    assert {k: ctx2.get_option(k) for k in keys} == opts


@pytest.mark.parametrize("claim", [1, 3, 4096])
def test_claim_sizes(gj, claim):
    """Waves of the fused propose kernel claiming 1, 3 or 4096 words of
    candidates at a time: counts and counters equal the depth-first path's."""
    src, dst = synth.rmat_draws(12, seed=7)
    n = 1 << 12
    ctx = gj.Context(0)
    ctx.set_option("batch_claim_words", claim)
    ctx.set_option("batch_heavy", 0)
    G = gj.Graph(ctx, src, dst, n)
    E = G.info()["edges"]
    reqs, _ = mixed_requests(gj, ctx, E, np.random.default_rng(claim), 24)
    counts, stats = gj.run_batch(ctx, G, reqs)
    for (q, lo, hi), c, st in zip(reqs, counts, stats):
        r = gj.count(ctx, G, q, lo, hi)
        assert c == r["matches"] and st["extensions"] == r["extensions"], (lo, hi)


@pytest.mark.parametrize("heavy", [0, 1, 2000])
def test_heavy_requests_split_off(gj, heavy):
    """Requests whose estimated work reaches batch_heavy run on the depth-first
    path and the rest fused (0: all fused; 1: every non-empty request
    depth-first; 2000: a mix): counts and counters equal the oracle's."""
    src, dst = synth.rmat_draws(11, seed=23)
    n = 1 << 11
    ctx = gj.Context(0)
    ctx.set_option("batch_heavy", heavy)
    assert ctx.get_option("batch_heavy") == heavy
    G = gj.Graph(ctx, src, dst, n)
    O = oracle.Graph(n, src, dst)
    reqs, specs = mixed_requests(gj, ctx, O.num_edges, np.random.default_rng(5), 36)
    counts, stats = gj.run_batch(ctx, G, reqs)
    for (q, lo, hi), c, st in zip(specs, counts, stats):
        ref = oracle.run(O, q, seed_lo=lo, seed_hi=hi)
        assert (c, st["prefixes"], st["extensions"]) == (ref["matches"], ref["prefixes"], ref["extensions"]), \
            (q, lo, hi)
    with pytest.raises(gj.GJError):
        ctx.set_option("batch_heavy", -1)
