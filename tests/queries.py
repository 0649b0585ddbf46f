"""Subgraph queries used by the tests: (num_attrs, atoms, global order).

An atom (s, d) is edge(a_s, a_d).  Attributes are 0-based (a1 -> 0).
"""
# transitive triangle e(a1,a2), e(a2,a3), e(a1,a3)   (evaluation query list, Sec. 5)
TRIANGLE = (3, [(0, 1), (1, 2), (0, 2)], [0, 1, 2])
# cyclic triangle e(a1,a2), e(a2,a3), e(a3,a1)        (Sec. 1.1, Appendix A)
CYCLIC_TRIANGLE = (3, [(0, 1), (1, 2), (2, 0)], [0, 1, 2])
# 4-clique: all six pairs i < j                        (evaluation query list, Sec. 5)
CLIQUE4 = (4, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)], [0, 1, 2, 3])
# diamond as two 2-paths a1->a2->a4, a1->a3->a4
DIAMOND = (4, [(0, 1), (0, 2), (1, 3), (2, 3)], [0, 1, 2, 3])
# diamond as printed in the evaluation query list: e(a1,a2), e(a2,a3), e(a4,a1), e(a4,a3)
PAPER_DIAMOND = (4, [(0, 1), (1, 2), (3, 0), (3, 2)], [0, 1, 2, 3])
# directed 4-cycle a1->a2->a3->a4->a1
CYCLE4 = (4, [(0, 1), (1, 2), (2, 3), (3, 0)], [0, 1, 2, 3])
# house (evaluation query list, Sec. 5)
HOUSE = (5, [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3), (1, 4), (2, 4)],
         [0, 1, 2, 3, 4])
# 5-clique
CLIQUE5 = (5, [(i, j) for i in range(5) for j in range(i + 1, 5)], [0, 1, 2, 3, 4])
# a query with a second atom over the first two attributes (a P_2 filter):
# reciprocal pair a1<->a2 closed by a3
RECIPROCAL = (3, [(0, 1), (1, 0), (1, 2), (2, 0)], [0, 1, 2])

ALL = {
    "triangle": TRIANGLE,
    "cyclic_triangle": CYCLIC_TRIANGLE,
    "clique4": CLIQUE4,
    "diamond": DIAMOND,
    "paper_diamond": PAPER_DIAMOND,
    "cycle4": CYCLE4,
    "house": HOUSE,
    "clique5": CLIQUE5,
    "reciprocal": RECIPROCAL,
}


def with_order(q, order):
    return (q[0], q[1], list(order))


def valid_orders(q):
    """Every global order whose first two attributes share an atom and whose
    later attributes each have an atom to an earlier one."""
    import itertools
    m, atoms, _ = q
    out = []
    for perm in itertools.permutations(range(m)):
        pos = {a: i for i, a in enumerate(perm)}
        ok = any(max(pos[s], pos[d]) == 1 for s, d in atoms)
        for j in range(2, m):
            ok = ok and any(max(pos[s], pos[d]) == j for s, d in atoms)
        if ok:
            out.append(list(perm))
    return out


# Symmetry breaking (Sec. 5.4): inequalities (x, y), value of a_x below a_y,
# that pick one match of every orbit of the query's automorphisms on an
# undirected (symmetric) input, with the size of that group.
SYM_LESS = {
    "triangle": ([(0, 1), (1, 2)], 6),
    "clique4": ([(0, 1), (1, 2), (2, 3)], 24),
    "clique5": ([(0, 1), (1, 2), (2, 3), (3, 4)], 120),
    # house: swapping a2, a3 or a1, a4 preserves it (each pair is adjacent)
    "house": ([(1, 2), (0, 3)], 4),
}


def with_less(q, less):
    return (q[0], q[1], list(q[2]), list(less))


# Queries whose last attributes share no atom, so counts factorise (Sec. 5.4):
# the house (trailing a4, a5), a 3-star (three out-neighbours of a1) and a fan
# (a path a1 -> a2 with two out-neighbours of a2).
STAR3 = (4, [(0, 1), (0, 2), (0, 3)], [0, 1, 2, 3])
FAN = (4, [(0, 1), (1, 2), (1, 3)], [0, 1, 2, 3])
FACTORISABLE = {"house": HOUSE, "star3": STAR3, "fan": FAN}


def trailing_run(q):
    """First position of the trailing run of attributes that share no atom and
    no inequality (at least two of them, after the seed pair), else 0."""
    m, atoms, order = q[0], q[1], q[2]
    less = q[3] if len(q) > 3 else []
    pairs = {frozenset(a) for a in atoms} | {frozenset(x) for x in less}
    j0 = m - 1
    while j0 - 1 >= 2 and all(frozenset((order[j0 - 1], order[t])) not in pairs for t in range(j0, m)):
        j0 -= 1
    return j0 if m - j0 >= 2 else 0


# Ternary atoms (Sec. 5.4): tri(x, y, z) is the triangle relation (x -> y,
# x -> z, y -> z), binding a_z after a_x and a_y.  The paper's 4-clique over
# three tri atoms (with the edge atom the seed pair comes from), a 5-clique
# over six, and a mixed query.
TRI_CLIQUE4 = (4, [(0, 1)], [0, 1, 2, 3], [], [(0, 1, 2), (0, 1, 3), (0, 2, 3)])
TRI_CLIQUE5 = (5, [(0, 1)], [0, 1, 2, 3, 4], [],
               [(0, 1, 2), (0, 1, 3), (0, 2, 3), (0, 1, 4), (0, 2, 4), (0, 3, 4)])
TRI_MIXED = (4, [(0, 1), (2, 3)], [0, 1, 2, 3], [], [(0, 1, 2)])
TRI = {"tri_clique4": TRI_CLIQUE4, "tri_clique5": TRI_CLIQUE5, "tri_mixed": TRI_MIXED}
