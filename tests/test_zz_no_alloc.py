"""The allocation-free count (gj_count_noalloc) against gj_run's count, to
the same bar as every count here (bit-exact counts and counters), through
the C ABI: two calls in a row, the second on a smaller input, for several
queries and batch bounds; a bound beyond the scratch is rejected."""
import ctypes

import numpy as np
import pytest

import synth
from tests import queries as Q

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gj():
    import paper_1802_03760_amd as gj
    return gj


def same(a, b):
    return (a["matches"], a["prefixes"], a["extensions"]) == (b["matches"], b["prefixes"], b["extensions"])


@pytest.mark.parametrize("name", ["triangle", "cyclic_triangle", "clique4", "diamond", "cycle4", "house",
                                  "reciprocal"])
def test_noalloc_equals_run(gj, name):
    q = Q.ALL[name]
    c = gj.Context(0)
    big_src, big_dst = synth.rmat_draws(13, seed=21)
    small_src, small_dst = synth.rmat_draws(10, seed=22)
    Gb = gj.Graph(c, big_src, big_dst, 1 << 13)
    Gs = gj.Graph(c, small_src, small_dst, 1 << 10)
    qh = gj.Query(c, *q)
    E = Gb.info(degrees=False)["edges"]
    width = 4000 if q[0] <= 3 else 400
    # first call: a slice of the larger graph; second: the whole smaller graph
    for G, lo, hi in ((Gb, E // 3, E // 3 + width), (Gs, 0, (1 << 64) - 1)):
        ref = gj.count(c, G, qh, lo, hi)
        got = gj.count_noalloc(c, G, qh, lo, hi)
        assert same(got, ref), (name, lo, hi, got["matches"], ref["matches"])
        assert got["kernel_ms"] == 0.0
    Gb.close()
    Gs.close()
    c.close()


def test_noalloc_small_bounds_many_batches(gj):
    """Batch bounds of 64 and 1024 prefixes: hundreds of proposal batches
    through the scratch, the larger input first."""
    c = gj.Context(0)
    src, dst = synth.rmat_draws(12, seed=5)
    G = gj.Graph(c, src, dst, 1 << 12)
    q = gj.Query(c, *Q.CLIQUE4)
    E = G.info(degrees=False)["edges"]
    for cap, (lo, hi) in ((1024, (0, 3000)), (64, (100, 900))):
        ref = gj.count(c, G, q, lo, hi)
        got = gj.count_noalloc(c, G, q, lo, hi, frontier_cap=cap)
        assert same(got, ref), cap
        assert got["kernel_launches"] > 10
    assert E > 3000
    G.close()
    c.close()


def test_noalloc_rejects_bound_beyond_scratch(gj):
    c = gj.Context(0)
    src, dst = synth.rmat_draws(8, seed=1)
    G = gj.Graph(c, src, dst, 1 << 8)
    q = gj.Query(c, *Q.TRIANGLE)
    for cap in (1 << 24, 32):
        with pytest.raises(gj.GJError) as e:
            gj.count_noalloc(c, G, q, frontier_cap=cap)
        assert e.value.status == gj.GJ_EINVAL and "frontier_cap" in str(e.value)
    # the context still works afterwards, through both entry points
    ref = gj.count(c, G, q)
    assert same(gj.count_noalloc(c, G, q), ref)
    G.close()
    c.close()


def test_noalloc_makes_no_allocation(gj):
    """With a counting allocator installed, the allocation-free count asks
    it for nothing (gj_run on the same context allocates its workspace)."""
    calls = []

    class Counting(gj.DeviceAllocator):
        def __init__(self):
            self.hip = ctypes.CDLL("libamdhip64.so")

        def alloc(self, nbytes, stream):
            p = ctypes.c_void_p()
            calls.append(nbytes)
            return p.value if self.hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes)) == 0 else 0

        def free(self, ptr, stream):
            self.hip.hipFree(ctypes.c_void_p(ptr))

    c = gj.Context(0, allocator=Counting())
    src, dst = synth.rmat_draws(11, seed=3)
    G = gj.Graph(c, src, dst, 1 << 11)
    q = gj.Query(c, *Q.CLIQUE4)
    n0 = len(calls)
    got = gj.count_noalloc(c, G, q)
    assert len(calls) == n0
    ref = gj.count(c, G, q)
    assert len(calls) > n0
    assert same(got, ref)
    G.close()
    c.close()
