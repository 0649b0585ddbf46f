"""CPU oracle for Generic Join subgraph queries -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously-correct C++ (gj_oracle.cpp) wrapped with ctypes.  Only
the tests, the smoke check and the CPU-baseline leg of the benchmark load it;
the GPU library never imports, links or calls anything here, and this package
shares no code with it.

Paper: Ammar, McSherry, Salihoglu, Joglekar, "Distributed Evaluation of
Subgraph Queries Using Worst-case Optimal Low-Memory Dataflows".  Generic Join
(Sec. 2.2, Fig. 1), its prefix-extension stage (Sec. 3.1, Sec. 4.1), the
edge-seeded dataflow (Sec. 4.2), Delta-GJ (Sec. 3.3.1) and the symmetry
breaking of Sec. 5.4 (inequality filters; vertices renamed by degree).

A query is (num_attrs, atoms, order[, less[, tris]]): less a list of (x, y)
meaning the value of a_x is below that of a_y; tris a list of (x, y, z), the
ternary atoms tri(a_x, a_y, a_z) (x -> y, x -> z and y -> z are edges) of
Sec. 5.4, each binding a_z after a_x and a_y.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gj_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

MAX_ATTRS = 8


class OracleError(RuntimeError):
    pass


def build():
    cmd = ["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-pthread", _SRC,
           "-o", _LIB + ".tmp"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        vp, u64, u32, i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_graph_new.restype = vp
        L.or_graph_new.argtypes = [u32, vp, vp, u64]
        L.or_graph_copy.restype = vp
        L.or_graph_copy.argtypes = [vp]
        L.or_graph_free.argtypes = [vp]
        L.or_graph_edges.restype = u64
        L.or_graph_edges.argtypes = [vp]
        L.or_graph_vertices.restype = u32
        L.or_graph_vertices.argtypes = [vp]
        L.or_graph_edge_list.argtypes = [vp, vp, vp]
        L.or_graph_noops.argtypes = [vp, vp, vp]
        L.or_query_valid.restype = i32
        L.or_query_valid.argtypes = [i32, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp, i32]
        L.or_run.restype = vp
        L.or_run.argtypes = [vp, i32, vp, vp, i32, vp, vp, vp, i32, vp, vp, vp, i32, i32, i32, u64, u64,
                             i32, ip]
        L.or_run_textbook.restype = vp
        L.or_run_textbook.argtypes = [vp, i32, vp, vp, i32, vp, vp, ip]
        L.or_delta.restype = vp
        L.or_delta.argtypes = [vp, vp, vp, vp, u64, i32, vp, vp, i32, vp, vp, vp, i32, i32, i32, ip]
        L.or_twopath.restype = i32
        L.or_twopath.argtypes = [vp, i32, i32, vp]
        L.or_result_matches.restype = u64
        L.or_result_matches.argtypes = [vp]
        L.or_result_counters.argtypes = [vp, vp, vp]
        L.or_result_num_rows.restype = u64
        L.or_result_num_rows.argtypes = [vp]
        L.or_result_rows.argtypes = [vp, vp]
        L.or_result_signs.argtypes = [vp, vp]
        L.or_result_count_delta.restype = ctypes.c_int64
        L.or_result_count_delta.argtypes = [vp]
        L.or_result_raw_emissions.restype = u64
        L.or_result_raw_emissions.argtypes = [vp]
        L.or_result_free.argtypes = [vp]
        _lib = L
    return _lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data) if a.size else None


def _query_arrays(query):
    num_attrs, atoms, order = query[:3]
    less = list(query[3]) if len(query) > 3 else []
    s = np.array([a for a, _ in atoms], dtype=np.uint8)
    d = np.array([b for _, b in atoms], dtype=np.uint8)
    o = np.array(order, dtype=np.uint8)
    lx = np.array([x for x, _ in less], dtype=np.uint8)
    ly = np.array([y for _, y in less], dtype=np.uint8)
    return num_attrs, s, d, len(atoms), o, lx, ly, len(less)


def _tri_arrays(query):
    tris = list(query[4]) if len(query) > 4 else []
    return tuple(np.array([t[i] for t in tris], dtype=np.uint8) for i in range(3)) + (len(tris),)


def query_valid(query):
    m, s, d, k, o, lx, ly, nl = _query_arrays(query)
    tx, ty, tz, nt = _tri_arrays(query)
    return bool(_load().or_query_valid(m, _p(s), _p(d), k, _p(o), _p(lx), _p(ly), nl,
                                       _p(tx), _p(ty), _p(tz), nt))


class Graph:
    """Edge relation: self-loops dropped, repeated edges collapsed."""

    def __init__(self, n, src, dst, _handle=None):
        L = _load()
        if _handle is not None:
            self._h = _handle
            return
        src = np.ascontiguousarray(src, dtype=np.uint32)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        self._h = L.or_graph_new(n, _p(src), _p(dst), len(src))
        if not self._h:
            raise OracleError("vertex id out of range")

    def __del__(self):
        if getattr(self, "_h", None) and _lib is not None:
            _lib.or_graph_free(self._h)
            self._h = None

    def copy(self):
        return Graph(0, None, None, _handle=_load().or_graph_copy(self._h))

    @property
    def num_edges(self):
        return int(_load().or_graph_edges(self._h))

    @property
    def num_vertices(self):
        return int(_load().or_graph_vertices(self._h))

    def edge_list(self):
        m = self.num_edges
        s = np.empty(m, dtype=np.uint32)
        d = np.empty(m, dtype=np.uint32)
        if m:
            _load().or_graph_edge_list(self._h, _p(s), _p(d))
        return s, d

    def noops(self):
        a = np.zeros(2, dtype=np.uint64)
        _load().or_graph_noops(self._h, ctypes.c_void_p(a.ctypes.data),
                               ctypes.c_void_p(a.ctypes.data + 8))
        return int(a[0]), int(a[1])


def _take(res, m, want_rows, want_signs=False, delta=False):
    L = _load()
    out = {"matches": int(L.or_result_matches(res))}
    pre = np.zeros(MAX_ATTRS + 1, dtype=np.uint64)
    ext = np.zeros(MAX_ATTRS + 1, dtype=np.uint64)
    L.or_result_counters(res, _p(pre), _p(ext))
    out["prefixes"] = [int(x) for x in pre]
    out["extensions"] = [int(x) for x in ext]
    n = int(L.or_result_num_rows(res))
    if want_rows:
        rows = np.empty((n, m), dtype=np.uint32)
        if n:
            L.or_result_rows(res, _p(rows))
        out["rows"] = rows
    if want_signs:
        sg = np.empty(n, dtype=np.int8)
        if n:
            L.or_result_signs(res, _p(sg))
        out["signs"] = sg
    if delta:
        out["count_delta"] = int(L.or_result_count_delta(res))
        out["raw_emissions"] = int(L.or_result_raw_emissions(res))
    L.or_result_free(res)
    return out


def run(graph, query, collect=False, seed_lo=0, seed_hi=None, threads=1, factorise=False):
    """Edge-seeded Generic Join; rows in attribute-index order, sorted.
    factorise: count a trailing run of independent attributes as a product
    of their extension counts (counts only)."""
    m, s, d, k, o, lx, ly, nl = _query_arrays(query)
    tx, ty, tz, nt = _tri_arrays(query)
    st = ctypes.c_int(0)
    hi = (1 << 64) - 1 if seed_hi is None else seed_hi
    res = _load().or_run(graph._h, m, _p(s), _p(d), k, _p(o), _p(lx), _p(ly), nl, _p(tx), _p(ty), _p(tz),
                         nt, int(collect), int(factorise), seed_lo, hi, threads, ctypes.byref(st))
    if st.value != 0:
        if res:
            _load().or_result_free(res)
        raise OracleError("or_run status %d" % st.value)
    return _take(res, m, collect)


def textbook(graph, query):
    """Textbook GJ from P_0; returns [P_1, ..., P_m] as position-order arrays
    (queries without inequalities)."""
    m, s, d, k, o, _, _, nl = _query_arrays(query)
    if nl or len(query) > 4:
        raise OracleError("textbook(): inequalities and ternary atoms are not supported")
    sizes = np.zeros(MAX_ATTRS + 2, dtype=np.uint64)
    st = ctypes.c_int(0)
    res = _load().or_run_textbook(graph._h, m, _p(s), _p(d), k, _p(o), _p(sizes),
                                  ctypes.byref(st))
    if st.value != 0:
        raise OracleError("or_run_textbook status %d" % st.value)
    L = _load()
    total = sum(int(sizes[j]) * j for j in range(1, m + 1))
    flat = np.empty(max(total, 1), dtype=np.uint32)
    if total:
        L.or_result_rows(res, _p(flat))
    L.or_result_free(res)
    out, off = [], 0
    for j in range(1, m + 1):
        n = int(sizes[j])
        out.append(flat[off:off + n * j].reshape(n, j))
        off += n * j
    return out


def delta(graph, src, dst, sign, query=None, rows=True, threads=1):
    """Applies the batch to `graph` in place; returns the query's delta.
    rows=False keeps only sums: count_delta (the signed sum of the outputs of
    every dQ_i), raw_emissions and the counters."""
    src = np.ascontiguousarray(src, dtype=np.uint32)
    dst = np.ascontiguousarray(dst, dtype=np.uint32)
    sign = np.ascontiguousarray(sign, dtype=np.int8)
    st = ctypes.c_int(0)
    if query is None:
        res = _load().or_delta(graph._h, _p(src), _p(dst), _p(sign), len(src),
                               0, None, None, 0, None, None, None, 0, 0, threads, ctypes.byref(st))
        m = 0
    else:
        if len(query) > 4 and query[4]:
            raise OracleError("delta(): ternary atoms are not supported")
        m, s, d, k, o, lx, ly, nl = _query_arrays(query)
        res = _load().or_delta(graph._h, _p(src), _p(dst), _p(sign), len(src),
                               m, _p(s), _p(d), k, _p(o), _p(lx), _p(ly), nl, int(rows), threads,
                               ctypes.byref(st))
    if st.value != 0:
        raise OracleError("or_delta status %d" % st.value)
    if query is None:
        _load().or_result_free(res)
        return None
    return _take(res, m, rows, rows, delta=True)


TWOPATH_KINDS = {"diamond": 0, "cycle4": 1}


def twopath(graph, kind, threads=1):
    """Counts of the diamond edge(a0,a1), edge(a0,a2), edge(a1,a3),
    edge(a2,a3) (kind "diamond") or the 4-cycle a0 -> a1 -> a2 -> a3 -> a0
    (kind "cycle4") by counting 2-paths, with the Generic Join counters of
    the order a0, a1, a2, a3 summed from their definitions.  Returns
    {"matches", "prefixes", "extensions"} shaped as run()'s."""
    out = np.zeros(6, dtype=np.uint64)
    st = _load().or_twopath(graph._h, TWOPATH_KINDS[kind], threads, _p(out))
    if st != 0:
        raise OracleError("or_twopath status %d" % st)
    pre = [0] * (MAX_ATTRS + 1)
    ext = [0] * (MAX_ATTRS + 1)
    pre[2], ext[2], pre[3], ext[3], pre[4] = (int(x) for x in out[1:6])
    return {"matches": int(out[0]), "prefixes": pre, "extensions": ext}


def symmetric_edges(n, src, dst):
    """Every distinct unordered pair {u, v}, u != v, of the input edges in
    both directions, sorted by (src, dst)."""
    s = np.asarray(src, dtype=np.int64)
    d = np.asarray(dst, dtype=np.int64)
    keep = s != d
    lo = np.minimum(s[keep], d[keep])
    hi = np.maximum(s[keep], d[keep])
    pairs = np.unique(lo * n + hi)
    a, b = pairs // n, pairs % n
    u = np.concatenate([a, b])
    v = np.concatenate([b, a])
    order = np.lexsort((v, u))
    return u[order].astype(np.uint32), v[order].astype(np.uint32)


def relabel_by_degree(n, src, dst, undirected=False):
    """The input transform of the symmetry-breaking optimisation (Sec. 5.4):
    the input is read as undirected (distinct unordered pairs {u, v}, u != v);
    vertex u's degree is the number of pairs that contain it; new ids are the
    ranks of the vertices by ascending degree, ties by ascending old id.  Each
    pair becomes the edge from its lower new id to its higher one, or both
    directions when `undirected`.  Returns (src, dst, old_of_new): the edges in
    new ids sorted by (src, dst), and the old id of every new id."""
    u, v = symmetric_edges(n, src, dst)
    deg = np.bincount(u.astype(np.int64), minlength=n)
    old_of_new = np.lexsort((np.arange(n), deg))  # primary key: degree
    new_of_old = np.empty(n, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(n)
    nu, nv = new_of_old[u], new_of_old[v]
    keep = np.ones(len(nu), dtype=bool) if undirected else nu < nv
    nu, nv = nu[keep], nv[keep]
    order = np.lexsort((nv, nu))
    return nu[order].astype(np.uint32), nv[order].astype(np.uint32), old_of_new.astype(np.uint32)
