"""MI355X Generic Join: Python binding of libgj.so (include/gj.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libgj.so.  PyTorch provides device memory and streams.  Importing
this package fails loudly when the library has not been built.
"""
import atexit
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgj.so")

GJ_OK, GJ_EINVAL, GJ_ENOMEM, GJ_EDEVICE, GJ_EOVERFLOW, GJ_EUNSUPPORTED, GJ_EBUSY = range(7)
MODE_COUNT, MODE_ENUMERATE = 0, 1
GJ_INPUT_DEVICE = 1
GJ_BUILD_UNDIRECTED, GJ_BUILD_DEGREE_ORDER = 4, 8
MAX_LESS = 28
MAX_ATTRS = 8
STATUS_NAMES = {0: "GJ_OK", 1: "GJ_EINVAL", 2: "GJ_ENOMEM", 3: "GJ_EDEVICE",
                4: "GJ_EOVERFLOW", 5: "GJ_EUNSUPPORTED", 6: "GJ_EBUSY"}

if not os.path.exists(LIB_PATH):
    raise ImportError("libgj.so is not built (run __graft_entry__.build() or "
                      "python paper_1802_03760_amd/build.py); there is no fallback")
_lib = ctypes.CDLL(LIB_PATH)

EXPORTS = ["gj_ctx_create", "gj_ctx_destroy", "gj_last_error", "gj_ctx_set_option", "gj_ctx_get_option",
           "gj_graph_build", "gj_graph_info", "gj_graph_csr", "gj_graph_destroy",
           "gj_query_register", "gj_query_destroy", "gj_run", "gj_apply_updates",
           "gj_last_delta", "gj_run_batch", "gj_autotune", "gj_server_create", "gj_server_submit_count",
           "gj_server_submit_update", "gj_server_wait", "gj_server_get_stats", "gj_server_destroy",
           "gj_server_set_option", "gj_query_register_ex", "gj_graph_vertex_ids", "gj_query_register_rel",
           "gj_graph_index_triangles", "gj_count_noalloc",
           "gj_measure_peaks"]
REQ_COUNT, REQ_UPDATE = 0, 1
SERVER_MAX_QUERIES = 16


class Atom(ctypes.Structure):
    _fields_ = [("src_attr", ctypes.c_uint8), ("dst_attr", ctypes.c_uint8)]


class Less(ctypes.Structure):
    _fields_ = [("lo_attr", ctypes.c_uint8), ("hi_attr", ctypes.c_uint8)]


class TriAtom(ctypes.Structure):
    _fields_ = [("x_attr", ctypes.c_uint8), ("y_attr", ctypes.c_uint8), ("z_attr", ctypes.c_uint8)]


class Tuning(ctypes.Structure):
    _fields_ = [("batch_lin", ctypes.c_uint32), ("batch_waves_per_cu", ctypes.c_uint32),
                ("batch_claim_words", ctypes.c_uint32), ("hash_index", ctypes.c_uint32),
                ("propose_u", ctypes.c_uint32), ("batch_heavy", ctypes.c_uint64),
                ("best_ms", ctypes.c_double), ("configs_tried", ctypes.c_int),
                ("from_cache", ctypes.c_int), ("batch_run", ctypes.c_uint32), ("run_ratio", ctypes.c_uint32)]


class ServerResult(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("status", ctypes.c_int), ("count", ctypes.c_uint64),
                ("nq", ctypes.c_uint32), ("count_delta", ctypes.c_int64 * 16),
                ("version", ctypes.c_uint64), ("batch_size", ctypes.c_uint32),
                ("submit_ns", ctypes.c_int64), ("start_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("completed_counts", ctypes.c_uint64), ("completed_updates", ctypes.c_uint64),
                ("count_batches", ctypes.c_uint64), ("mean_count_batch", ctypes.c_double),
                ("count_p50_ms", ctypes.c_double), ("count_p99_ms", ctypes.c_double),
                ("update_p50_ms", ctypes.c_double), ("update_p99_ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("matches", ctypes.c_uint64),
                ("prefixes", ctypes.c_uint64 * (MAX_ATTRS + 1)),
                ("extensions", ctypes.c_uint64 * (MAX_ATTRS + 1)),
                ("noop_inserts", ctypes.c_uint64),
                ("noop_deletes", ctypes.c_uint64),
                ("raw_emissions", ctypes.c_uint64),
                ("kernel_launches", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double),
                ("ms", ctypes.c_double)]

    def as_dict(self):
        return {"matches": int(self.matches),
                "prefixes": [int(x) for x in self.prefixes],
                "extensions": [int(x) for x in self.extensions],
                "noop_inserts": int(self.noop_inserts),
                "noop_deletes": int(self.noop_deletes),
                "raw_emissions": int(self.raw_emissions),
                "kernel_launches": int(self.kernel_launches),
                "kernel_ms": float(self.kernel_ms),
                "ms": float(self.ms)}


_vp, _u64, _u32, _i32 = ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int
# gj_allocator: device memory callbacks (include/gj.h)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class AllocatorStruct(ctypes.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("free", FREE_FN), ("user", ctypes.c_void_p)]


_lib.gj_ctx_create.argtypes = [_i32, _vp, ctypes.POINTER(AllocatorStruct), ctypes.POINTER(_vp)]
_lib.gj_ctx_create.restype = _i32
_lib.gj_ctx_destroy.argtypes = [_vp]
_lib.gj_ctx_destroy.restype = None
_lib.gj_last_error.argtypes = [_vp]
_lib.gj_last_error.restype = ctypes.c_char_p
_lib.gj_ctx_set_option.argtypes = [_vp, ctypes.c_char_p, ctypes.c_int64]
_lib.gj_ctx_set_option.restype = _i32
_lib.gj_ctx_get_option.argtypes = [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)]
_lib.gj_ctx_get_option.restype = _i32
_lib.gj_graph_build.argtypes = [_vp, _vp, _vp, _u64, _u32, _u32, ctypes.POINTER(_vp)]
_lib.gj_graph_build.restype = _i32
_lib.gj_graph_info.argtypes = [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u32),
                               ctypes.POINTER(_u32), ctypes.POINTER(_u32), ctypes.POINTER(_u64)]
_lib.gj_graph_info.restype = _i32
_lib.gj_graph_csr.argtypes = [_vp, _i32, ctypes.POINTER(_vp), ctypes.POINTER(_vp), ctypes.POINTER(_vp)]
_lib.gj_graph_csr.restype = _i32
_lib.gj_graph_destroy.argtypes = [_vp]
_lib.gj_graph_destroy.restype = None
_lib.gj_query_register.argtypes = [_vp, _u32, ctypes.POINTER(Atom), _u32, _vp, ctypes.POINTER(_vp)]
_lib.gj_query_register.restype = _i32
_lib.gj_query_register_ex.argtypes = [_vp, _u32, ctypes.POINTER(Atom), _u32, _vp, ctypes.POINTER(Less), _u32,
                                      ctypes.POINTER(_vp)]
_lib.gj_query_register_ex.restype = _i32
_lib.gj_query_register_rel.argtypes = [_vp, _u32, ctypes.POINTER(Atom), _u32, ctypes.POINTER(TriAtom), _u32, _vp,
                                       ctypes.POINTER(Less), _u32, ctypes.POINTER(_vp)]
_lib.gj_query_register_rel.restype = _i32
_lib.gj_graph_index_triangles.argtypes = [_vp, _vp, ctypes.POINTER(_u64)]
_lib.gj_graph_index_triangles.restype = _i32
_lib.gj_graph_vertex_ids.argtypes = [_vp, _vp, _i32]
_lib.gj_graph_vertex_ids.restype = _i32
_lib.gj_query_destroy.argtypes = [_vp]
_lib.gj_query_destroy.restype = None
_lib.gj_run.argtypes = [_vp, _vp, _vp, _i32, _u64, _u64, _vp, _u64, _i32, ctypes.POINTER(Stats)]
_lib.gj_run.restype = _i32
_lib.gj_measure_peaks.argtypes = [_vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
_lib.gj_measure_peaks.restype = _i32
_lib.gj_count_noalloc.argtypes = [_vp, _vp, _vp, _u64, _u64, _u64, ctypes.POINTER(Stats)]
_lib.gj_count_noalloc.restype = _i32
_lib.gj_apply_updates.argtypes = [_vp, _vp, _vp, _vp, _vp, _u64, _i32, ctypes.POINTER(_vp), _u32,
                                  _vp, ctypes.POINTER(_vp), ctypes.POINTER(_vp), _vp, _vp,
                                  ctypes.POINTER(Stats)]
_lib.gj_apply_updates.restype = _i32
_lib.gj_last_delta.argtypes = [_vp, _u32, _vp, _vp, _u64, _i32, ctypes.POINTER(_u64)]
_lib.gj_last_delta.restype = _i32
_lib.gj_server_create.argtypes = [_vp, _vp, _u32, _u64, ctypes.POINTER(_vp)]
_lib.gj_server_create.restype = _i32
_lib.gj_server_submit_count.argtypes = [_vp, _vp, _u64, _u64, ctypes.POINTER(_u64)]
_lib.gj_server_submit_count.restype = _i32
_lib.gj_server_submit_update.argtypes = [_vp, _vp, _vp, _vp, _u64, ctypes.POINTER(_vp), _u32,
                                         ctypes.POINTER(_u64)]
_lib.gj_server_submit_update.restype = _i32
_lib.gj_server_wait.argtypes = [_vp, _u64, ctypes.c_int64, ctypes.POINTER(ServerResult)]
_lib.gj_server_wait.restype = _i32
_lib.gj_server_set_option.argtypes = [_vp, ctypes.c_char_p, ctypes.c_int64]
_lib.gj_server_set_option.restype = _i32
_lib.gj_server_get_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
_lib.gj_server_get_stats.restype = _i32
_lib.gj_server_destroy.argtypes = [_vp]
_lib.gj_server_destroy.restype = None
_lib.gj_run_batch.argtypes = [_vp, _vp, _u32, ctypes.POINTER(_vp), _vp, _vp, _vp, ctypes.POINTER(Stats)]
_lib.gj_run_batch.restype = _i32
_lib.gj_autotune.argtypes = [_vp, _vp, _u32, ctypes.POINTER(_vp), _vp, _vp, ctypes.c_char_p,
                             ctypes.POINTER(Tuning)]
_lib.gj_autotune.restype = _i32


class _Handle:
    """A library handle plus the handles that must be released before it.

    The records live apart from the Python objects that own them and hold
    their dependants strongly, so a handle is never destroyed before what
    was built on it, whatever order finalisers run in.  (When the garbage
    collector frees a reference cycle it clears weak references first and
    then calls __del__ in no particular order.)"""

    __slots__ = ("h", "destroy", "deps", "parents", "keep")

    def __init__(self, h, destroy, parents=(), keep=None):
        self.h, self.destroy, self.deps, self.parents = h, destroy, {}, []
        self.keep = keep  # kept alive until the handle is destroyed (e.g. allocator callbacks)
        for p in parents:
            self.depend(p)

    def depend(self, parent):
        """Release self before parent."""
        if parent.h is not None and id(self) not in parent.deps:
            parent.deps[id(self)] = self
            self.parents.append(parent)

    def close(self):
        if self.h is None:
            return
        for d in list(self.deps.values()):
            d.close()
        h, self.h = self.h, None
        self.destroy(h)
        self.keep = None
        for p in self.parents:
            p.deps.pop(id(self), None)
        self.parents = []


# Context handles still open; at interpreter exit each is released, with
# everything built on it, while the HIP runtime is still fully up.
# Afterwards the finalisers do nothing.
_roots = {}
_finalised = False


def _release_all():
    global _finalised
    for hd in list(_roots.values()):
        hd.close()
    _roots.clear()
    _finalised = True


atexit.register(_release_all)


class _Owner:
    """Base of the handle-owning wrappers: close() releases the handle and
    everything that depends on it; __del__ does the same until exit."""

    _hd = None

    @property
    def _h(self):
        return self._hd.h if self._hd is not None else None

    def close(self):
        if self._hd is not None:
            self._hd.close()

    def __del__(self):
        if not _finalised:
            self.close()


class GJError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


def _np_ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None and a.size else None


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr(x):
    """Device or host address of a torch tensor / numpy array."""
    if x is None:
        return None
    if _is_torch(x):
        return ctypes.c_void_p(x.data_ptr()) if x.numel() else None
    return _np_ptr(x)


class DeviceAllocator:
    """Device memory source of a context (gj_allocator).  Subclasses define
    alloc(nbytes, stream) -> device address (0 when out of memory) and
    free(ptr, stream); the library calls free only after its stream has
    finished with the memory.  Exceptions in a callback count as a failed
    allocation (alloc) or are dropped (free)."""

    def alloc(self, nbytes, stream):
        raise NotImplementedError

    def free(self, ptr, stream):
        raise NotImplementedError

    def struct(self):
        if getattr(self, "_struct", None) is None:
            def a(user, nbytes, stream):
                try:
                    return int(self.alloc(int(nbytes), stream or 0) or 0)
                except Exception:
                    return 0

            def f(user, ptr, stream):
                try:
                    self.free(int(ptr), stream or 0)
                except Exception:
                    pass
            self._cb = (ALLOC_FN(a), FREE_FN(f))
            self._struct = AllocatorStruct(self._cb[0], self._cb[1], None)
        return self._struct


class TorchAllocator(DeviceAllocator):
    """Device memory from PyTorch's caching allocator, on the library's
    stream."""

    def __init__(self, device=0):
        import torch
        self.torch = torch
        self.device = device

    def alloc(self, nbytes, stream):
        return self.torch.cuda.caching_allocator_alloc(nbytes, self.device, int(stream))

    def free(self, ptr, stream):
        self.torch.cuda.caching_allocator_delete(ptr)


class Context(_Owner):
    """gj_ctx on one HIP device; issues work on `stream` (a torch.cuda.Stream,
    a raw hipStream_t int, or None for the library's own stream) and takes
    device memory from `allocator` (a DeviceAllocator, "torch" for
    PyTorch's caching allocator, or None for hipMalloc)."""

    def __init__(self, device=0, stream=None, allocator=None):
        h = _vp()
        raw = None
        if stream is not None:
            raw = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        if allocator == "torch":
            allocator = TorchAllocator(device)
        ap = ctypes.byref(allocator.struct()) if allocator is not None else None
        st = _lib.gj_ctx_create(device, _vp(raw) if raw else None, ap, ctypes.byref(h))
        if st != GJ_OK:
            raise GJError(st, "gj_ctx_create(device=%d) failed" % device)
        self.allocator = allocator
        self._hd = _Handle(h, _lib.gj_ctx_destroy, keep=allocator)
        self.device = device
        _roots[id(self._hd)] = self._hd

    def check(self, st, what):
        if st != GJ_OK:
            raise GJError(st, "%s: %s" % (what, _lib.gj_last_error(self._h).decode()))

    def set_option(self, key, value):
        self.check(_lib.gj_ctx_set_option(self._h, key.encode(), int(value)), "set_option")

    def get_option(self, key):
        v = ctypes.c_int64()
        self.check(_lib.gj_ctx_get_option(self._h, key.encode(), ctypes.byref(v)), "get_option")
        return v.value

    def close(self):
        """Destroys the context and every server, graph and query created on it."""
        hd = self._hd
        if hd is not None:
            hd.close()
            _roots.pop(id(hd), None)


class Graph(_Owner):
    """Forward and reverse CSR indexes of an edge list (gj_graph_build).
    undirected: store every distinct pair both ways; degree_order: rename
    vertices by degree and keep each pair once, lower new id to higher (both
    ways if undirected too) -- see vertex_ids()."""

    def __init__(self, ctx, src, dst, num_vertices, undirected=False, degree_order=False):
        self.ctx = ctx
        self.num_vertices = num_vertices
        h = _vp()
        if _is_torch(src):
            flags = GJ_INPUT_DEVICE if src.is_cuda else 0
            m = src.numel()
        else:
            src = np.ascontiguousarray(src, dtype=np.uint32)
            dst = np.ascontiguousarray(dst, dtype=np.uint32)
            flags, m = 0, len(src)
        flags |= (GJ_BUILD_UNDIRECTED if undirected else 0) | (GJ_BUILD_DEGREE_ORDER if degree_order else 0)
        ctx.check(_lib.gj_graph_build(ctx._h, _ptr(src), _ptr(dst), m, num_vertices, flags,
                                      ctypes.byref(h)), "gj_graph_build")
        self._hd = _Handle(h, _lib.gj_graph_destroy, (ctx._hd,))

    def info(self, degrees=True):
        """Edges, vertices and version; with degrees, the largest out- and
        in-degree too (which merges rows appended by log-structured updates)."""
        e, n, mo, mi, v = _u64(), _u32(), _u32(), _u32(), _u64()
        self.ctx.check(_lib.gj_graph_info(self._h, ctypes.byref(e), ctypes.byref(n),
                                          ctypes.byref(mo) if degrees else None,
                                          ctypes.byref(mi) if degrees else None, ctypes.byref(v)),
                       "gj_graph_info")
        out = {"edges": e.value, "vertices": n.value, "version": v.value}
        if degrees:
            out.update(max_out=mo.value, max_in=mi.value)
        return out

    def index_triangles(self):
        """Builds the triangle relation for ternary atoms (gj_graph_index_triangles);
        returns its size."""
        t = _u64()
        self.ctx.check(_lib.gj_graph_index_triangles(self.ctx._h, self._h, ctypes.byref(t)),
                       "gj_graph_index_triangles")
        return t.value

    def vertex_ids(self):
        """Old id of every vertex id (gj_graph_vertex_ids), a numpy array."""
        out = np.empty(self.num_vertices, dtype=np.uint32)
        self.ctx.check(_lib.gj_graph_vertex_ids(self._h, _np_ptr(out), 0), "gj_graph_vertex_ids")
        return out

    def csr_ptrs(self, reverse=False):
        rp, col, row = _vp(), _vp(), _vp()
        self.ctx.check(_lib.gj_graph_csr(self._h, int(reverse), ctypes.byref(rp), ctypes.byref(col),
                                         ctypes.byref(row)), "gj_graph_csr")
        return rp.value, col.value, row.value



class Query(_Owner):
    """Q(a_0..a_{m-1}) := edge(s, d), ... with a global order, optional
    inequalities less = [(x, y), ...] (value of a_x below that of a_y) and
    ternary atoms tris = [(x, y, z), ...] over the triangle relation
    (gj_query_register_rel)."""

    def __init__(self, ctx, num_attrs, atoms, order=None, less=(), tris=()):
        self.ctx = ctx
        self.num_attrs = num_attrs
        self.atoms = [tuple(a) for a in atoms]
        self.order = list(range(num_attrs)) if order is None else list(order)
        self.less = [tuple(x) for x in less]
        arr = (Atom * len(self.atoms))(*[Atom(s, d) for s, d in self.atoms])
        lt = (Less * max(len(self.less), 1))(*[Less(x, y) for x, y in self.less])
        self.tris = [tuple(t) for t in tris]
        tr = (TriAtom * max(len(self.tris), 1))(*[TriAtom(*t) for t in self.tris])
        o = np.array(self.order, dtype=np.uint8)
        h = _vp()
        ctx.check(_lib.gj_query_register_rel(ctx._h, num_attrs, arr, len(self.atoms), tr, len(self.tris),
                                             _np_ptr(o), lt, len(self.less), ctypes.byref(h)),
                  "gj_query_register_rel")
        self._hd = _Handle(h, _lib.gj_query_destroy, (ctx._hd,))


def count(ctx, graph, query, seed_lo=0, seed_hi=(1 << 64) - 1):
    st = Stats()
    ctx.check(_lib.gj_run(ctx._h, graph._h, query._h, MODE_COUNT, seed_lo, seed_hi, None, 0, 0,
                          ctypes.byref(st)), "gj_run(count)")
    return st.as_dict()


class Server(_Owner):
    """Request server over a context and a graph (gj_server_*): its worker
    threads own both until close().  iteration_work, versions: server options
    (None keeps the library default)."""

    def __init__(self, ctx, graph, max_batch=64, mem_budget_bytes=0, iteration_work=None, versions=None):
        self.ctx, self.graph = ctx, graph
        h = _vp()
        st = _lib.gj_server_create(ctx._h, graph._h, max_batch, mem_budget_bytes, ctypes.byref(h))
        if st != GJ_OK:
            raise GJError(st, "gj_server_create")
        # Released before the context, the graph and every query it was sent.
        self._hd = _Handle(h, _lib.gj_server_destroy, (ctx._hd, graph._hd))
        self._keep = {}  # queries referenced by queued requests
        if iteration_work is not None:
            self.set_option("iteration_work", iteration_work)
        if versions is not None:
            self.set_option("versions", versions)

    def set_option(self, key, value):
        st = _lib.gj_server_set_option(self._h, key.encode(), int(value))
        if st != GJ_OK:
            raise GJError(st, "gj_server_set_option(%s)" % key)

    def submit_count(self, query, seed_lo=0, seed_hi=(1 << 64) - 1):
        t = _u64()
        st = _lib.gj_server_submit_count(self._h, query._h, seed_lo, seed_hi, ctypes.byref(t))
        if st != GJ_OK:
            raise GJError(st, "gj_server_submit_count")
        self._hd.depend(query._hd)
        self._keep[t.value] = query
        return t.value

    def submit_update(self, src, dst, sign, queries):
        src = np.ascontiguousarray(src, dtype=np.uint32)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        sign = np.ascontiguousarray(sign, dtype=np.int8)
        qh = (_vp * max(len(queries), 1))(*[q._h.value for q in queries])
        t = _u64()
        st = _lib.gj_server_submit_update(self._h, _np_ptr(src), _np_ptr(dst), _np_ptr(sign), len(src), qh,
                                          len(queries), ctypes.byref(t))
        if st != GJ_OK:
            raise GJError(st, "gj_server_submit_update")
        for q in queries:
            self._hd.depend(q._hd)
        self._keep[t.value] = list(queries)
        return t.value

    def wait(self, ticket, timeout_ms=-1):
        r = ServerResult()
        st = _lib.gj_server_wait(self._h, ticket, timeout_ms, ctypes.byref(r))
        if st != GJ_OK:
            raise GJError(st, "gj_server_wait")
        self._keep.pop(ticket, None)
        return {"kind": r.kind, "status": r.status, "count": int(r.count),
                "count_delta": [int(r.count_delta[i]) for i in range(r.nq)], "version": int(r.version),
                "batch_size": int(r.batch_size), "latency_ms": (r.done_ns - r.submit_ns) * 1e-6,
                "queue_ms": (r.start_ns - r.submit_ns) * 1e-6, "service_ms": (r.done_ns - r.start_ns) * 1e-6,
                "submit_ns": int(r.submit_ns), "start_ns": int(r.start_ns), "done_ns": int(r.done_ns)}

    def stats(self):
        s = ServerStats()
        _lib.gj_server_get_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in ServerStats._fields_}



def _requests(requests):
    n = len(requests)
    qh = (_vp * max(n, 1))(*[q._h.value for q, _, _ in requests])
    lo = np.array([int(l) for _, l, _ in requests] or [0], dtype=np.uint64)
    hi = np.array([int(h) for _, _, h in requests] or [0], dtype=np.uint64)
    return n, qh, lo, hi


def run_batch(ctx, graph, requests):
    """Counts of [(query, seed_lo, seed_hi), ...] in one fused, graph-captured
    pipeline (gj_run_batch).  Returns (counts, per-request stats)."""
    n, qh, lo, hi = _requests(requests)
    counts = np.zeros(max(n, 1), dtype=np.uint64)
    stats = (Stats * max(n, 1))()
    ctx.check(_lib.gj_run_batch(ctx._h, graph._h, n, qh, _np_ptr(lo), _np_ptr(hi), _np_ptr(counts), stats),
              "gj_run_batch")
    return [int(x) for x in counts[:n]], [stats[i].as_dict() for i in range(n)]


def autotune(ctx, graph, requests, cache_path=None):
    n, qh, lo, hi = _requests(requests)
    out = Tuning()
    ctx.check(_lib.gj_autotune(ctx._h, graph._h, n, qh, _np_ptr(lo), _np_ptr(hi),
                               cache_path.encode() if cache_path else None, ctypes.byref(out)),
              "gj_autotune")
    return {"batch_lin": out.batch_lin, "batch_waves_per_cu": out.batch_waves_per_cu,
            "batch_claim_words": out.batch_claim_words, "hash_index": out.hash_index,
            "propose_u": out.propose_u, "batch_heavy": out.batch_heavy, "batch_run": out.batch_run,
            "run_ratio": out.run_ratio, "best_ms": out.best_ms, "configs_tried": out.configs_tried,
            "from_cache": bool(out.from_cache)}


def enumerate_rows(ctx, graph, query, seed_lo=0, seed_hi=(1 << 64) - 1, out=None, cap=None):
    """Sorted match rows (attribute order).  `out`: a torch int32 cuda tensor of
    shape (cap, m) to write into, or a numpy uint32 host array; None sizes a host
    array from a count pass.  Returns (stats, rows)."""
    m = query.num_attrs
    if out is None:
        if cap is None:
            cap = count(ctx, graph, query, seed_lo, seed_hi)["matches"]
        out = np.empty((max(cap, 1), m), dtype=np.uint32)
    on_dev = 1 if (_is_torch(out) and out.is_cuda) else 0
    cap = out.shape[0] if cap is None else cap
    st = Stats()
    s = _lib.gj_run(ctx._h, graph._h, query._h, MODE_ENUMERATE, seed_lo, seed_hi, _ptr(out), cap,
                    on_dev, ctypes.byref(st))
    ctx.check(s, "gj_run(enumerate)")
    return st.as_dict(), out[: st.matches]


def measure_peaks(ctx):
    """gj_measure_peaks: measured device-copy and LDS bandwidth (GB/s)."""
    cp, lds = ctypes.c_double(), ctypes.c_double()
    ctx.check(_lib.gj_measure_peaks(ctx._h, ctypes.byref(cp), ctypes.byref(lds)), "gj_measure_peaks")
    return {"copy_gbs": cp.value, "lds_gbs": lds.value}


def count_noalloc(ctx, graph, query, seed_lo=0, seed_hi=(1 << 64) - 1, frontier_cap=0):
    """gj_count_noalloc: the count of gj_run on the depth-first path, every
    workspace buffer taken from the library's static scratch (no device
    allocation).  Returns the stats dict."""
    st = Stats()
    ctx.check(_lib.gj_count_noalloc(ctx._h, graph._h, query._h, seed_lo, seed_hi, frontier_cap,
                                    ctypes.byref(st)), "gj_count_noalloc")
    return st.as_dict()


def apply_updates(ctx, graph, src, dst, sign, queries, rows=False, cap=1 << 16):
    """Applies one signed batch; per query returns count_delta, and with
    rows=True the consolidated (rows, signs) as host arrays (fetched again with
    gj_last_delta when they outgrow the first buffer of `cap` rows)."""
    on_dev = 1 if (_is_torch(src) and src.is_cuda) else 0
    if not _is_torch(src):
        src = np.ascontiguousarray(src, dtype=np.uint32)
        dst = np.ascontiguousarray(dst, dtype=np.uint32)
        sign = np.ascontiguousarray(sign, dtype=np.int8)
    b = src.numel() if _is_torch(src) else len(src)
    nq = len(queries)
    qh = (_vp * max(nq, 1))(*[q._h.value for q in queries])
    cd = np.zeros(max(nq, 1), dtype=np.int64)
    nd = np.zeros(max(nq, 1), dtype=np.uint64)
    stats = (Stats * max(nq, 1))()
    row_bufs, sign_bufs = [], []
    rp = sp = capa = None
    if rows:
        if on_dev:
            raise ValueError("rows=True needs a host batch in this binding")
        capa = np.array([cap] * nq, dtype=np.uint64)
        for q in queries:
            row_bufs.append(np.empty((max(cap, 1), q.num_attrs), dtype=np.uint32))
            sign_bufs.append(np.empty(max(cap, 1), dtype=np.int8))
        rp = (_vp * nq)(*[r.ctypes.data for r in row_bufs])
        sp = (_vp * nq)(*[s.ctypes.data for s in sign_bufs])
    s = _lib.gj_apply_updates(ctx._h, graph._h, _ptr(src), _ptr(dst), _ptr(sign), b, on_dev, qh, nq,
                              _np_ptr(cd), rp, sp, _np_ptr(capa), _np_ptr(nd), stats)
    if not (rows and s == GJ_EOVERFLOW):
        ctx.check(s, "gj_apply_updates")
    out = []
    for i in range(nq):
        r = {"count_delta": int(cd[i]), "n_delta": int(nd[i]), "stats": stats[i].as_dict()}
        if rows:
            k = int(nd[i])
            if k > cap:
                row_bufs[i] = np.empty((k, queries[i].num_attrs), dtype=np.uint32)
                sign_bufs[i] = np.empty(k, dtype=np.int8)
                got = _u64()
                ctx.check(_lib.gj_last_delta(ctx._h, i, _np_ptr(row_bufs[i]), _np_ptr(sign_bufs[i]), k, 0,
                                             ctypes.byref(got)), "gj_last_delta")
            r["rows"] = row_bufs[i][:k]
            r["signs"] = sign_bufs[i][:k]
        out.append(r)
    return out


def last_delta(ctx, q_index, num_attrs, cap):
    """Rows and signs kept from the last apply_updates for query position q_index."""
    rows = np.empty((max(cap, 1), num_attrs), dtype=np.uint32)
    signs = np.empty(max(cap, 1), dtype=np.int8)
    got = _u64()
    ctx.check(_lib.gj_last_delta(ctx._h, q_index, _np_ptr(rows), _np_ptr(signs), cap, 0,
                                 ctypes.byref(got)), "gj_last_delta")
    return rows[: got.value], signs[: got.value]
