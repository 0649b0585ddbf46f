"""Owner-grouped first-stage kernel (counting triangles and cyclic triangles
over all seed edges): parity with the oracle and with the generic
per-candidate kernel on skewed, tied and segmented inputs."""
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
def ctxs(gj):
    auto = gj.Context(0)
    generic = gj.Context(0)
    generic.set_option("strategy", 1)
    return auto, generic


def both(gj, ctxs, n, src, dst, q):
    ref = oracle.run(oracle.Graph(n, src, dst), q, threads=8)
    out = []
    for c in ctxs:
        G = gj.Graph(c, src, dst, n)
        r = gj.count(c, G, gj.Query(c, *q))
        assert r["matches"] == ref["matches"], (q, r["matches"], ref["matches"])
        assert r["extensions"] == ref["extensions"]
        assert r["prefixes"] == ref["prefixes"]
        out.append(r)
    return ref


@pytest.mark.parametrize("scale", [13, 15])
@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle"])
def test_rmat(gj, ctxs, scale, name):
    src, dst = synth.rmat_draws(scale, seed=scale)
    ref = both(gj, ctxs, 1 << scale, src, dst, Q.ALL[name])
    assert ref["matches"] > 0


def test_equal_degrees_circulant(gj, ctxs):
    """i -> i+1 .. i+100 (mod n): every set has 100 elements, every
    count-minimisation is a tie.  n = 250 so that three offsets can sum to n
    (cyclic triangles exist)."""
    n, k = 250, 100
    i = np.repeat(np.arange(n), k)
    j = (i + np.tile(np.arange(1, k + 1), n)) % n
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE):
        assert both(gj, ctxs, n, i.astype(np.uint32), j.astype(np.uint32), q)["matches"] > 0


def test_hub_segments(gj, ctxs):
    """Hubs of out- and in-degree 30,000 (several table segments), leaves
    linked to random other leaves."""
    n = 30001
    rng = np.random.default_rng(3)
    leaves = np.arange(1, n, dtype=np.uint32)
    extra_s = rng.integers(1, n, 200000).astype(np.uint32)
    extra_d = rng.integers(1, n, 200000).astype(np.uint32)
    src = np.concatenate([np.zeros(n - 1, np.uint32), leaves, extra_s])
    dst = np.concatenate([leaves, np.zeros(n - 1, np.uint32), extra_d])
    for q in (Q.TRIANGLE, Q.CYCLIC_TRIANGLE):
        assert both(gj, ctxs, n, src, dst, q)["matches"] > 0


def test_complete_digraph(gj, ctxs):
    n = 90
    s, d = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = s != d
    ref = both(gj, ctxs, n, s[keep].astype(np.uint32), d[keep].astype(np.uint32), Q.TRIANGLE)
    assert ref["matches"] == n * (n - 1) * (n - 2)


def test_reverse_seed_order(gj, ctxs):
    """Order (a2, a1, a3): the seed atom edge(a1, a2) is read from the
    reverse index."""
    src, dst = synth.rmat_draws(12, seed=9)
    both(gj, ctxs, 1 << 12, src, dst, Q.with_order(Q.TRIANGLE, [1, 0, 2]))
    both(gj, ctxs, 1 << 12, src, dst, Q.with_order(Q.CYCLIC_TRIANGLE, [2, 0, 1]))
