"""Small named graphs for closed-form checks (edge lists only)."""
from __future__ import annotations

import itertools

import numpy as np


def complete(n):
    return n, list(itertools.combinations(range(n), 2))


def path(n):
    return n, [(i, i + 1) for i in range(n - 1)]


def cycle(n):
    return n, [(i, (i + 1) % n) for i in range(n)]


def star(n):
    """Centre 0 with n-1 leaves."""
    return n, [(0, i) for i in range(1, n)]


def wheel(m):
    """Hub 0 joined to every vertex of the cycle 1..m."""
    rim = [(1 + i, 1 + (i + 1) % m) for i in range(m)]
    return m + 1, rim + [(0, 1 + i) for i in range(m)]


def complete_bipartite(a, b):
    return a + b, [(i, a + j) for i in range(a) for j in range(b)]


def petersen():
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return 10, outer + spokes + inner


def grid(r, c):
    e = []
    for i in range(r):
        for j in range(c):
            v = i * c + j
            if j + 1 < c:
                e.append((v, v + 1))
            if i + 1 < r:
                e.append((v, v + c))
    return r * c, e


def random_tree(n, rng):
    return n, [(i, int(rng.integers(0, i))) for i in range(1, n)]


def random_graph(n, p, rng):
    e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < p]
    return n, e


def disjoint_union(g1, g2):
    n1, e1 = g1
    n2, e2 = g2
    return n1 + n2, list(e1) + [(u + n1, v + n1) for u, v in e2]


def relabel(g, perm):
    n, e = g
    return n, [(int(perm[u]), int(perm[v])) for u, v in e]


def dense(g):
    n, e = g
    A = np.zeros((n, n), dtype=np.int64)
    for u, v in e:
        if u != v:
            A[u, v] = A[v, u] = 1
    return A
