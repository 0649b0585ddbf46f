"""Brute-force subgraph matching by the definition: every vertex tuple that
satisfies every atom (join semantics).  Independent of the oracle: numpy over
all n^m tuples, for tiny graphs only."""
import numpy as np


def adjacency(n, src, dst):
    A = np.zeros((n, n), dtype=bool)
    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    keep = src != dst
    A[src[keep], dst[keep]] = True
    return A


def matches(A, query):
    """query = (m, atoms, order[, less[, tris]]); (x, y) in less requires the
    value of a_x to be below that of a_y; (x, y, z) in tris requires the
    edges x -> y, x -> z and y -> z."""
    m, atoms = query[0], query[1]
    less = query[3] if len(query) > 3 else []
    tris = query[4] if len(query) > 4 else []
    n = A.shape[0]
    T = np.indices((n,) * m).reshape(m, -1)  # lexicographic order
    ok = np.ones(T.shape[1], dtype=bool)
    for s, d in atoms:
        ok &= A[T[s], T[d]]
    for x, y in less:
        ok &= T[x] < T[y]
    for x, y, z in tris:  # tri(x, y, z): x -> y, x -> z, y -> z
        ok &= A[T[x], T[y]] & A[T[x], T[z]] & A[T[y], T[z]]
    return T[:, ok].T.astype(np.uint32)


def as_set(rows):
    return set(map(tuple, np.asarray(rows).tolist()))
