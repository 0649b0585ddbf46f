"""Device memory through the caller's allocator (gj_allocator of
gj_ctx_create): every allocation of a graph build, counts, enumeration,
update batches, the fused batch path and a server goes through the
callbacks and is returned exactly once; PyTorch's caching allocator serves
as one; and an allocation that fails at any point of those calls returns
GJ_ENOMEM and leaves the graph intact (counts and later updates still equal
the oracle's)."""
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


def counting_allocator(gj, fail_at=None):
    """hipMalloc / hipFree behind the callbacks, counting calls; the
    allocation numbered fail_at (1-based) returns NULL."""
    hip = ctypes.CDLL("libamdhip64.so")

    class Counting(gj.DeviceAllocator):
        def __init__(self):
            self.n = 0
            self.live = {}
            self.freed_twice = 0
            self.failed = 0

        def alloc(self, nbytes, stream):
            self.n += 1
            if fail_at is not None and self.n == fail_at:
                self.failed += 1
                return 0
            p = ctypes.c_void_p()
            if hip.hipMalloc(ctypes.byref(p), ctypes.c_size_t(nbytes)) != 0:
                return 0
            self.live[p.value] = nbytes
            return p.value

        def free(self, ptr, stream):
            if ptr not in self.live:
                self.freed_twice += 1
                return
            del self.live[ptr]
            hip.hipFree(ctypes.c_void_p(ptr))

    return Counting()


def workload(scale=11, seed=4):
    src, dst = synth.rmat_draws(scale, seed=seed)
    batch = synth.update_batch(scale, seed, 16 << scale, 9, 0, 3000)
    return 1 << scale, src, dst, batch


def test_every_allocation_through_callbacks(gj):
    n, src, dst, (bs, bd, bg) = workload()
    O = oracle.Graph(n, src, dst)
    A = counting_allocator(gj)
    c = gj.Context(0, allocator=A)
    G = gj.Graph(c, src, dst, n)
    assert A.n > 0 and A.live
    built = A.n
    tri, k4 = gj.Query(c, *Q.TRIANGLE), gj.Query(c, *Q.CLIQUE4)
    assert gj.count(c, G, tri)["matches"] == oracle.run(O, Q.TRIANGLE)["matches"]
    st, rows = gj.enumerate_rows(c, G, tri)
    assert np.array_equal(rows, oracle.run(O, Q.TRIANGLE, collect=True)["rows"])
    E = G.info(degrees=False)["edges"]
    reqs = [(k4, 0, 50), (tri, 100, 900), (k4, E // 2, E // 2 + 300)]
    counts, _ = gj.run_batch(c, G, reqs)
    assert counts == [oracle.run(O, q, seed_lo=lo, seed_hi=hi)["matches"]
                      for q, lo, hi in ((Q.CLIQUE4, 0, 50), (Q.TRIANGLE, 100, 900),
                                        (Q.CLIQUE4, E // 2, E // 2 + 300))]
    ref = oracle.delta(O, bs, bd, bg, Q.TRIANGLE)
    got = gj.apply_updates(c, G, bs, bd, bg, [tri], rows=True)[0]
    assert got["count_delta"] == ref["count_delta"] and np.array_equal(got["rows"], ref["rows"])
    srv = gj.Server(c, G)
    t = srv.submit_count(k4, 0, 200)
    assert srv.wait(t)["count"] == oracle.run(O, Q.CLIQUE4, seed_lo=0, seed_hi=200)["matches"]
    srv.close()
    assert A.n > built
    G.close()
    c.close()
    assert not A.live, "allocations never returned: %d" % len(A.live)
    assert A.freed_twice == 0


def test_torch_allocator(gj):
    import torch
    n, src, dst, (bs, bd, bg) = workload(12, 6)
    O = oracle.Graph(n, src, dst)
    before = torch.cuda.memory_allocated(0)
    c = gj.Context(0, stream=torch.cuda.current_stream(), allocator="torch")
    G = gj.Graph(c, src, dst, n)
    q = gj.Query(c, *Q.TRIANGLE)
    assert gj.count(c, G, q)["matches"] == oracle.run(O, Q.TRIANGLE)["matches"]
    assert torch.cuda.memory_allocated(0) > before + 16 * G.info(degrees=False)["edges"]
    r = gj.apply_updates(c, G, bs, bd, bg, [q])[0]
    assert r["count_delta"] == oracle.delta(O, bs, bd, bg, Q.TRIANGLE, rows=False)["count_delta"]
    assert gj.count(c, G, q)["matches"] == oracle.run(O, Q.TRIANGLE)["matches"]
    G.close()
    c.close()
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated(0) == before


def test_failure_at_every_allocation(gj):
    """For every allocation number N of the sequence build, triangle count,
    4-clique slice count, enumeration, fused batch, update batch: the call
    that reaches allocation N fails with GJ_ENOMEM; retried (the allocator
    fails only once) it succeeds, and every later result equals the
    oracle's -- a failed update leaves the graph as it was."""
    n, src, dst, (bs, bd, bg) = workload(10, 8)
    O0 = oracle.Graph(n, src, dst)
    c_tri = oracle.run(O0, Q.TRIANGLE)["matches"]
    c_k4 = oracle.run(O0, Q.CLIQUE4, seed_lo=0, seed_hi=400)
    rows0 = oracle.run(O0, Q.TRIANGLE, collect=True)["rows"]
    O1 = O0.copy()
    d_ref = oracle.delta(O1, bs, bd, bg, Q.TRIANGLE)
    c_tri1 = oracle.run(O1, Q.TRIANGLE)["matches"]
    # number of allocations of the whole sequence, from a run without failures
    total = None
    N = 1
    while total is None or N <= total:
        A = counting_allocator(gj, fail_at=N)
        c = gj.Context(0, allocator=A)
        c.set_option("delta_fused", 1)
        failures = []

        def attempt(f, what):
            try:
                return f()
            except gj.GJError as e:
                assert e.status == gj.GJ_ENOMEM, (N, what, e)
                failures.append(what)
                return f()

        G = attempt(lambda: gj.Graph(c, src, dst, n), "build")
        tri = gj.Query(c, *Q.TRIANGLE)
        k4 = gj.Query(c, *Q.CLIQUE4)
        assert attempt(lambda: gj.count(c, G, tri), "count")["matches"] == c_tri, N
        r = attempt(lambda: gj.count(c, G, k4, 0, 400), "slice")
        assert (r["matches"], r["extensions"]) == (c_k4["matches"], c_k4["extensions"]), N
        st, rows = attempt(lambda: gj.enumerate_rows(c, G, tri), "enumerate")
        assert np.array_equal(rows, rows0), N
        counts, _ = attempt(lambda: gj.run_batch(c, G, [(k4, 0, 400), (tri, 0, 300)]), "batch")
        assert counts[0] == c_k4["matches"], N
        info0 = G.info()

        def update():
            return gj.apply_updates(c, G, bs, bd, bg, [tri], rows=True)[0]
        try:
            d = update()
        except gj.GJError as e:
            assert e.status == gj.GJ_ENOMEM, (N, e)
            failures.append("update")
            # the failed batch changed nothing
            assert G.info() == info0, N
            assert gj.count(c, G, tri)["matches"] == c_tri, N
            d = update()
        assert d["count_delta"] == d_ref["count_delta"] and np.array_equal(d["rows"], d_ref["rows"]), N
        # the first count of the new version plans its owner tasks (an allocation)
        assert attempt(lambda: gj.count(c, G, tri), "count after update")["matches"] == c_tri1, N
        G.close()
        c.close()
        assert not A.live and A.freed_twice == 0, N
        if total is None:
            total = A.n  # the first pass (N = 1) fails the build's first allocation
            assert failures == ["build"]
        else:
            assert len(failures) == (1 if A.failed else 0), (N, failures)
        N += 1
    assert total > 10
