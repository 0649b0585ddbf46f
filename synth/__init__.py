"""Seeded synthetic inputs: R-MAT and Erdos-Renyi edge lists, update batches.

Input generation only: nothing here dedupes, indexes or joins.  The GPU
library and the CPU oracle both take these raw arrays and normalise them on
their own.  The C source (synth.c) is compiled by :func:`build`.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None

# R-MAT quadrant probabilities used for every synthetic workload here
RMAT_ABC = (0.57, 0.19, 0.19)


def build():
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", _SRC,
           "-o", _LIB + ".tmp", "-lm"]
    subprocess.check_call(cmd)
    os.replace(_LIB + ".tmp", _LIB)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        u64, u32, dbl, i32 = (ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_double, ctypes.c_int)
        vp = ctypes.c_void_p
        lib.synth_splitmix64.restype = u64
        lib.synth_splitmix64.argtypes = [u64, u64]
        lib.synth_rmat.restype = None
        lib.synth_rmat.argtypes = [i32, u64, u64, dbl, dbl, dbl, u64, i32, vp, vp]
        lib.synth_er.restype = u64
        lib.synth_er.argtypes = [u32, u64, u64, vp, vp]
        lib.synth_batch_size.restype = u64
        lib.synth_batch_size.argtypes = [u64, u64, u64, u64]
        lib.synth_update_batch.restype = u64
        lib.synth_update_batch.argtypes = [i32, dbl, dbl, dbl, u64, u64, u64,
                                           u64, u64, dbl, vp, vp, vp]
        _lib = lib
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data)


def splitmix64(key, n):
    return int(_load().synth_splitmix64(key, n))


def rmat_draws(scale, edge_factor=16, seed=0, first=0, count=None,
               abc=RMAT_ABC, threads=None):
    """Raw R-MAT draws (duplicates and self-loops kept) as (src, dst) uint32."""
    if count is None:
        count = edge_factor << scale
    threads = threads or min(16, os.cpu_count() or 1)
    src = np.empty(count, dtype=np.uint32)
    dst = np.empty(count, dtype=np.uint32)
    a, b, c = abc
    _load().synth_rmat(scale, first, count, a, b, c, seed, threads,
                       _ptr(src), _ptr(dst))
    return src, dst


def er_edges(n, m, seed=0):
    """m distinct loop-free arcs over n vertices as (src, dst) uint32."""
    src = np.empty(m, dtype=np.uint32)
    dst = np.empty(m, dtype=np.uint32)
    if _load().synth_er(n, m, seed, _ptr(src), _ptr(dst)) == 0 and m:
        raise ValueError("cannot draw %d distinct arcs over %d vertices" % (m, n))
    return src, dst


def batch_size(seed, k, lo, hi):
    return int(_load().synth_batch_size(seed, k, lo, hi))


def update_batch(scale, base_seed, base_draws, seed, k, size, del_frac=0.1,
                 abc=RMAT_ABC):
    """Signed update batch k: (src, dst, sign int8 in {+1,-1})."""
    src = np.empty(max(size, 1), dtype=np.uint32)
    dst = np.empty(max(size, 1), dtype=np.uint32)
    sign = np.empty(max(size, 1), dtype=np.int8)
    a, b, c = abc
    n = _load().synth_update_batch(scale, a, b, c, base_seed, base_draws, seed,
                                   k, size, del_frac, _ptr(src), _ptr(dst),
                                   _ptr(sign))
    return src[:n].copy(), dst[:n].copy(), sign[:n].copy()


def update_stream(scale, base_seed, seed, n_batches, lo, hi, del_frac=0.1,
                  edge_factor=16, abc=RMAT_ABC):
    """Yields (k, src, dst, sign) for batches 0..n_batches-1 with log-uniform sizes."""
    base_draws = edge_factor << scale
    for k in range(n_batches):
        size = batch_size(seed, k, lo, hi)
        s, d, g = update_batch(scale, base_seed, base_draws, seed, k, size,
                               del_frac, abc)
        yield k, s, d, g
