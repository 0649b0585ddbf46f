"""The C ABI library loads and exports every function include/gj.h declares
(CPU only: no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    txt = open(os.path.join(ROOT, "include", "gj.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gj_[a-z_]+)\s*\(", txt)))


def test_exports_match_header():
    import paper_1802_03760_amd as gj
    lib = ctypes.CDLL(gj.LIB_PATH)
    names = declared()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(gj.EXPORTS) == names


def test_struct_layout():
    import paper_1802_03760_amd as gj
    # uint64 matches + 2 x 9 uint64 + 4 uint64 + 2 double
    assert ctypes.sizeof(gj.Stats) == 8 * (1 + 18 + 4 + 2)
    assert ctypes.sizeof(gj.Atom) == 2


def test_no_oracle_in_product():
    """The library and its binding never reach the oracle."""
    pkg = os.path.join(ROOT, "paper_1802_03760_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                t = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in t.replace("Oracle", ""), f


def _fake_tree(log):
    """Handles shaped like a context, a graph, a query and a server on them,
    whose destroy functions only record the order of release."""
    import paper_1802_03760_amd as gj
    rel = lambda name: (lambda h: log.append(name))
    c = gj._Handle(1, rel("ctx"))
    g = gj._Handle(2, rel("graph"), (c,))
    q = gj._Handle(3, rel("query"), (c,))
    s = gj._Handle(4, rel("server"), (c, g))
    s.depend(q)
    return c, g, q, s


def _check_order(log):
    assert sorted(log) == ["ctx", "graph", "query", "server"]
    assert log.index("server") < log.index("graph") < log.index("ctx")
    assert log.index("server") < log.index("query") < log.index("ctx")


def test_release_order_from_any_handle():
    """Closing any handle first releases what depends on it, each handle once."""
    for first in range(4):
        log = []
        hs = _fake_tree(log)
        hs[first].close()
        for h in hs:
            h.close()
        _check_order(log)
        assert all(not h.deps for h in hs)


def test_release_order_in_a_collected_cycle():
    """Wrappers freed together by the cycle collector (which clears weak
    references before any finaliser runs, in no fixed order) still release
    servers before queries and graphs, and those before their context."""
    import gc
    import paper_1802_03760_amd as gj

    class W(gj._Owner):
        def __init__(self, hd, *refs):
            self._hd, self.refs = hd, list(refs)

    for perm in range(6):
        log = []
        c, g, q, s = _fake_tree(log)
        objs = [W(c), W(g), W(q), W(s)]
        for o in objs[1:]:
            o.refs.append(objs[0])
        objs[3].refs += [objs[1], objs[2]]
        objs[0].refs.append(objs[3 - perm % 4])   # close a cycle through the context
        objs[perm % 4].refs.append(objs)          # and one through a list
        del c, g, q, s, o, objs
        gc.collect()
        _check_order(log)


def test_device_memory_only_through_dev_alloc():
    """Device memory is taken in one place, which uses the context's
    allocator when one was given (gj_allocator); the only other device
    buffer is the allocation-free path's static scratch array."""
    csrc = os.path.join(ROOT, "paper_1802_03760_amd", "csrc")
    sites = []
    for f in sorted(os.listdir(csrc)):
        t = open(os.path.join(csrc, f)).read()
        for name in ("hipMalloc(", "hipMallocAsync(", "hipExtMallocWithFlags(", "hipMallocManaged("):
            sites += [f] * t.count(name)
    assert sites == ["api.hip"]
    api = open(os.path.join(csrc, "api.hip")).read()
    start = api.index("void* dev_alloc(gj_ctx* c, size_t bytes)")
    assert api.index("hipMalloc(") > start and api.index("hipMalloc(") < api.index("void dev_free(")
