"""GPU parity of factorised counts (Sec. 5.4; the "factorise" option of
gj_run counts) against the CPU oracle's factorised evaluation: counts and
every per-stage counter, on R-MAT graphs, with inequalities, over seed
slices and with frontier caps small enough to split the work into many
batches; and equality with the plain (enumerating) count."""
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


def _ctx(gj, **opts):
    c = gj.Context(0)
    c.set_option("factorise", 1)
    for k, v in opts.items():
        c.set_option(k, v)
    return c


@pytest.mark.parametrize("name", sorted(Q.FACTORISABLE))
def test_factorised_parity(gj, name):
    c, cp = _ctx(gj), gj.Context(0)
    assert c.get_option("factorise") == 1 and cp.get_option("factorise") == 0
    src, dst = synth.rmat_draws(10, seed=21)
    n = 1 << 10
    G, Gp, O = gj.Graph(c, src, dst, n), gj.Graph(cp, src, dst, n), oracle.Graph(n, src, dst)
    q0 = Q.FACTORISABLE[name]
    rng = np.random.default_rng(3)
    orders = Q.valid_orders(q0)
    done = 0
    for order in orders[:: max(1, len(orders) // 4)][:4]:
        for less in ([], [tuple(rng.choice(q0[0], 2, replace=False).tolist())]):
            q = Q.with_less(Q.with_order(q0, order), less)
            ref = oracle.run(O, q, factorise=True, threads=8)
            r = gj.count(c, G, gj.Query(c, *q))
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), q
            assert gj.count(cp, Gp, gj.Query(cp, *q))["matches"] == ref["matches"]
            done += Q.trailing_run(q) > 0
    assert done > 0


def test_factorised_small_batches_and_slices(gj):
    """Tiny seed chunks and frontier caps (hundreds of prefix batches reach
    the trailing run) and seed slices give the oracle's counts."""
    c = _ctx(gj, frontier_cap=64, seed_chunk=100)
    src, dst = synth.rmat_draws(9, seed=22)
    n = 1 << 9
    G, O = gj.Graph(c, src, dst, n), oracle.Graph(n, src, dst)
    E = G.info()["edges"]
    for name in ("house", "star3", "fan"):
        q = Q.FACTORISABLE[name]
        h = gj.Query(c, *q)
        for lo, hi in ((0, E), (0, 1), (E // 3, E // 3 + 700), (E - 5, E + 10)):
            ref = oracle.run(O, q, factorise=True, seed_lo=lo, seed_hi=hi)
            r = gj.count(c, G, h, lo, hi)
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), (name, lo, hi)


def test_factorised_edge_cases(gj):
    """Empty graph; a graph where a trailing attribute never extends (a
    single edge); a star (one trailing set huge, products large)."""
    c = _ctx(gj)
    n = 3001
    leaves = np.arange(1, n, dtype=np.uint32)
    cases = [(np.array([], np.uint32), np.array([], np.uint32), 4),
             (np.array([0], np.uint32), np.array([1], np.uint32), 2),
             (np.concatenate([np.zeros(n - 1, np.uint32), leaves]),
              np.concatenate([leaves, np.zeros(n - 1, np.uint32)]), n)]
    for s, d, nv in cases:
        G, O = gj.Graph(c, s, d, nv), oracle.Graph(nv, s, d)
        for q in Q.FACTORISABLE.values():
            ref = oracle.run(O, q, factorise=True, threads=8)
            r = gj.count(c, G, gj.Query(c, *q))
            assert (r["matches"], r["prefixes"], r["extensions"]) == \
                (ref["matches"], ref["prefixes"], ref["extensions"]), (nv, q)
    with pytest.raises(gj.GJError):
        c.set_option("factorise", 2)
