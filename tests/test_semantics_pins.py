"""Pins of the dense GraphBLAS-semantics oracle (Section III) against hand
worked examples, textbook reductions and the paper's algorithms run end to
end through it."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
from oracle import semantics as S
import graphs as G


def mat_from_dense(D, present=None, kind="int64"):
    present = (D != 0) if present is None else present
    e = {(int(i), int(j)): (D[i, j].item() if kind != "bool" else 1)
         for i, j in zip(*np.nonzero(present))}
    return S.Mat(D.shape[0], D.shape[1], e, kind)


def adj_mat(g):
    n, e = g
    A = G.dense(g)
    return S.Mat(n, n, {(int(i), int(j)): 1 for i, j in zip(*np.nonzero(A))}, "bool")


# ------------------------------------------------------- worked examples

def test_write_rules_worked_by_hand():
    w = S.Vec(4, {0: 10, 1: 20, 3: 40}, "int64")
    m = S.Vec(4, {0: 1, 1: 0, 2: 1}, "int64")
    u = S.Vec(4, {1: 100, 2: 200, 3: 300}, "int64")
    assert S.assign_vector(w, m, None, u).e == {1: 20, 2: 200, 3: 40}
    assert S.assign_vector(w, m, None, u, replace=True).e == {2: 200}
    assert S.assign_vector(w, m, "plus", u).e == {0: 10, 1: 20, 2: 200, 3: 40}
    assert S.assign_vector(w, m, None, u, struct=True).e == {1: 100, 2: 200, 3: 40}
    assert S.assign_vector(w, m, None, u, struct=True, comp=True).e == {0: 10, 1: 20, 3: 300}
    assert S.assign_vector(w, m, None, u, struct=True, comp=True, replace=True).e == {3: 300}
    assert S.assign_vector(w, None, "plus", u).e == {0: 10, 1: 120, 2: 200, 3: 340}
    assert S.assign_vector(w, None, None, u, comp=True).e == w.e
    assert S.assign_vector(w, None, None, u, comp=True, replace=True).e == {}


def test_semirings_worked_by_hand():
    A = S.Mat(2, 3, {(0, 0): 1, (0, 1): 1, (1, 1): 1, (1, 2): 1}, "bool")
    B = S.Mat(3, 2, {(0, 0): 1, (1, 0): 1, (1, 1): 1, (2, 1): 1}, "bool")
    C = S.Mat(2, 2, {}, "int64")
    assert S.mxm(C, None, None, "plus.pair", A, B).e == {(0, 0): 2, (0, 1): 1, (1, 0): 1, (1, 1): 2}
    T = S.mxm(C, None, None, "any.secondi", A, B).e
    assert T[(0, 0)].c == {0, 1} and T[(0, 1)] == 1 and T[(1, 0)] == 1 and T[(1, 1)].c == {1, 2}
    Td = S.mxm(C, None, None, "any.secondi", A, B, deterministic=True).e
    assert Td == {(0, 0): 0, (0, 1): 1, (1, 0): 1, (1, 1): 1}
    Av = S.Mat(2, 3, {(0, 0): 2.0, (0, 1): 3.0, (1, 1): 5.0, (1, 2): 7.0}, "fp64")
    Bv = S.Mat(3, 2, {(0, 0): 1.0, (1, 0): 10.0, (1, 1): 0.5, (2, 1): 4.0}, "fp64")
    Cf = S.Mat(2, 2, {}, "fp64")
    assert S.mxm(Cf, None, None, "plus.first", Av, Bv).e == {(0, 0): 5.0, (0, 1): 3.0, (1, 0): 5.0, (1, 1): 12.0}
    assert S.mxm(Cf, None, None, "min.plus", Av, Bv).e == {(0, 0): 3.0, (0, 1): 3.5, (1, 0): 15.0, (1, 1): 5.5}
    # complemented structural mask + replace, as in the BFS step
    M = S.Mat(2, 2, {(0, 0): 0}, "int64")
    out = S.mxm(S.Mat(2, 2, {(1, 0): 9}, "int64"), M, None, "plus.pair", A, B,
                comp=True, struct=True, replace=True).e
    assert out == {(0, 1): 1, (1, 0): 1, (1, 1): 2}


# -------------------------------------------------- textbook reductions

def test_plus_pair_is_integer_product_on_patterns():
    rng = np.random.default_rng(0)
    for shape in [(5, 7, 4), (8, 8, 8), (3, 9, 6)]:
        m, k, n = shape
        Ad = (rng.random((m, k)) < 0.4).astype(np.int64)
        Bd = (rng.random((k, n)) < 0.4).astype(np.int64)
        P = Ad @ Bd
        T = S.mxm(S.Mat(m, n, {}, "int64"), None, None, "plus.pair",
                  mat_from_dense(Ad, kind="bool"), mat_from_dense(Bd, kind="bool")).e
        assert T == {(int(i), int(j)): int(P[i, j]) for i, j in zip(*np.nonzero(P))}
        # transposes through the descriptor equal explicit transposes
        T2 = S.mxm(S.Mat(m, n, {}, "int64"), None, None, "plus.pair",
                   mat_from_dense(Ad.T.copy(), kind="bool"), mat_from_dense(Bd.T.copy(), kind="bool"),
                   tran0=True, tran1=True).e
        assert T2 == T


def test_plus_first_is_value_product_with_ones():
    rng = np.random.default_rng(1)
    Ad = rng.integers(-5, 6, size=(6, 5)).astype(np.float64)
    pres = rng.random((6, 5)) < 0.5
    Ad = np.where(pres, Ad, 0.0)
    Bp = rng.random((5, 4)) < 0.5
    T = S.mxm(S.Mat(6, 4, {}, "fp64"), None, None, "plus.first",
              mat_from_dense(Ad, present=pres, kind="fp64"),
              mat_from_dense(Bp.astype(np.int64), kind="bool")).e
    want = Ad @ Bp.astype(np.float64)
    cnt = pres.astype(int) @ Bp.astype(int)
    assert T == {(int(i), int(j)): float(want[i, j]) for i, j in zip(*np.nonzero(cnt))}


def test_min_plus_one_hot_and_bellman_ford_and_dijkstra():
    rng = np.random.default_rng(4)
    n = 12
    W = np.where(rng.random((n, n)) < 0.25, rng.integers(1, 10, size=(n, n)), 0).astype(np.float64)
    np.fill_diagonal(W, 0)
    A = mat_from_dense(W, kind="fp64")
    # one-hot u times A is row s of A shifted by u(s)
    u = S.Vec(n, {3: 2.5}, "fp64")
    r = S.vxm(S.Vec(n, {}, "fp64"), None, None, "min.plus", u, A).e
    assert r == {int(j): 2.5 + W[3, j] for j in np.nonzero(W[3])[0]}
    # k rounds of t = min(t, t min.plus A) equal k rounds of Bellman-Ford
    src = 0
    t = S.Vec(n, {src: 0.0}, "fp64")
    bf = np.full(n, np.inf)
    bf[src] = 0.0
    edges = [(i, j, W[i, j]) for i, j in zip(*np.nonzero(W))]
    for _ in range(n):
        t = S.vxm(t, None, "min", "min.plus", t, A)
        nb = bf.copy()
        for i, j, w in edges:
            if bf[i] + w < nb[j]:
                nb[j] = bf[i] + w
        bf = nb
        got = np.full(n, np.inf)
        for j, x in t.e.items():
            got[j] = x
        assert np.array_equal(got, bf)
    D = csg.dijkstra(sp.csr_matrix(W), directed=True, indices=src)
    assert np.array_equal(got, D)


def test_reduce_and_ewise_against_numpy():
    rng = np.random.default_rng(9)
    D = rng.integers(1, 20, size=(6, 7))
    pres = rng.random((6, 7)) < 0.5
    A = mat_from_dense(np.where(pres, D, 0), present=pres)
    w = S.reduce_rows(S.Vec(6, {}, "int64"), None, None, "plus", A)
    assert w.e == {i: int(D[i][pres[i]].sum()) for i in range(6) if pres[i].any()}
    w = S.reduce_rows(S.Vec(7, {}, "int64"), None, None, "min", A, tran0=True)
    assert w.e == {j: int(D[:, j][pres[:, j]].min()) for j in range(7) if pres[:, j].any()}
    assert S.reduce_scalar(A, "plus") == int(D[pres].sum())
    pres2 = rng.random((6, 7)) < 0.5
    B = mat_from_dense(np.where(pres2, 2 * D, 0), present=pres2)
    C0 = S.Mat(6, 7, {}, "int64")
    add = S.ewise_add(C0, None, None, "plus", A, B).e
    mul = S.ewise_mult(C0, None, None, "times", A, B).e
    for i in range(6):
        for j in range(7):
            a = D[i, j] if pres[i, j] else None
            b = 2 * D[i, j] if pres2[i, j] else None
            if a is None and b is None:
                assert (i, j) not in add
            else:
                assert add[(i, j)] == (a or 0) + (b or 0)
            if a is not None and b is not None:
                assert mul[(i, j)] == a * b
            else:
                assert (i, j) not in mul


# ------------------------------------- the paper's algorithms through it

def alg1_bfs(A: S.Mat, s: int):
    n = A.nrows
    p = S.Vec(n, {s: s}, "int64")
    q = S.Vec(n, {s: s}, "int64")
    level = {s: 0}
    for lev in range(1, n):
        q = S.vxm(q, p, None, "any.secondi", q, A, comp=True, struct=True, replace=True)
        p = S.assign_vector(p, q, None, q, struct=True)
        for v in q.e:
            level[v] = lev
        if not q.e:
            break
    return level, p


def test_algorithm1_through_semantics_matches_queue_bfs():
    rng = np.random.default_rng(21)
    for n, pr in [(15, 0.2), (20, 0.12)]:
        g = G.random_graph(n, pr, rng)
        A = adj_mat(g)
        rp, ci = oracle.from_edges(*g)
        for s in (0, n - 1):
            level, p = alg1_bfs(A, s)
            lv, pa = oracle.bfs(rp, ci, s)
            assert {v: int(lv[v]) for v in range(n) if lv[v] >= 0} == level
            for v, cand in p.e.items():
                if v == s:
                    assert cand == s
                    continue
                cs = cand.c if isinstance(cand, S.AnyOf) else {cand}
                assert cs == {u for u in ci[rp[v]:rp[v + 1]] if lv[u] == lv[v] - 1}
                assert pa[v] in cs


def alg3_bc(A: S.Mat, sources):
    """Algorithm 3 with the backtrack running i = d down to 1."""
    n, ns = A.nrows, len(sources)
    P = S.Mat(ns, n, {(k, int(s)): 1.0 for k, s in enumerate(sources)}, "fp64")
    F = S.mxm(S.Mat(ns, n, {}, "fp64"), P, None, "plus.first", P, A, comp=True, struct=True)
    Sd = []
    while True:
        Sd.append(S.Mat(ns, n, {k: 1 for k in F.e}, "bool"))
        P = S.ewise_add(P, None, None, "plus", P, F)
        F = S.mxm(F, P, None, "plus.first", F, A, comp=True, struct=True, replace=True)
        if not F.e:
            break
    d = len(Sd) - 1
    B = S.Mat(ns, n, {(k, j): 1.0 for k in range(ns) for j in range(n)}, "fp64")
    W = S.Mat(ns, n, {}, "fp64")
    for i in range(d, 0, -1):
        W = S.ewise_mult(W, Sd[i], None, "div", B, P, struct=True, replace=True)
        W = S.mxm(W, Sd[i - 1], None, "plus.first", W, A, struct=True, replace=True, tran1=True)
        B = S.ewise_mult(B, None, "plus", "times", W, P)
    cent = np.full(n, -float(ns))
    for (k, j), v in B.e.items():
        cent[j] += v
    return cent


def test_algorithm3_through_semantics_matches_brandes():
    rng = np.random.default_rng(8)
    for g in [G.path(6), G.star(6), G.random_graph(14, 0.25, rng), G.random_graph(16, 0.18, rng)]:
        n = g[0]
        A = adj_mat(g)
        rp, ci = oracle.from_edges(*g)
        srcs = [0, n // 2, n - 1]
        assert np.allclose(alg3_bc(A, srcs), oracle.brandes(rp, ci, srcs), rtol=1e-12, atol=1e-9)


def test_algorithm6_through_semantics_matches_oracle():
    rng = np.random.default_rng(6)
    g = G.random_graph(18, 0.35, rng)
    A = adj_mat(g)
    L = S.strictly_lower(A)
    U = S.Mat(A.nrows, A.ncols, {k: v for k, v in A.e.items() if k[1] > k[0]}, "bool")
    C1 = S.mxm(S.Mat(A.nrows, A.ncols, {}, "int64"), L, None, "plus.pair", L, U,
               struct=True, tran1=True)
    C2 = S.mxm(S.Mat(A.nrows, A.ncols, {}, "int64"), L, None, "plus.pair", L, L,
               struct=True, tran1=True)
    t = oracle.triangle_count(*oracle.from_edges(*g))
    assert S.reduce_scalar(C1, "plus") == t == S.reduce_scalar(C2, "plus")
    lrp, lci, cnt = oracle.lower_counts(*oracle.from_edges(*g))
    rows = np.repeat(np.arange(A.nrows), np.diff(lrp))
    assert C2.e == {(int(i), int(j)): int(c) for i, j, c in zip(rows, lci, cnt) if c > 0}


def test_algorithm5_fixpoint_through_semantics_matches_dijkstra():
    """min.plus relaxation to a fixpoint (what delta-stepping computes, bucket
    by bucket) through the brute-force semantics equals the Dijkstra oracle."""
    import graphgen
    rng = np.random.default_rng(8)
    n = 14
    rp, ci = oracle.from_edges(n, G.random_graph(n, 0.3, rng)[1])
    w = graphgen.edge_weights(rp, ci, 8, 20)
    W = np.zeros((n, n))
    for u in range(n):
        W[u, ci[rp[u]:rp[u + 1]]] = w[rp[u]:rp[u + 1]]
    A = mat_from_dense(W, kind="fp64")
    t = S.Vec(n, {0: 0.0}, "fp64")
    for _ in range(n):
        t = S.vxm(t, None, "min", "min.plus", t, A)
    got = np.full(n, np.inf)
    for j, x in t.e.items():
        got[j] = x
    assert np.array_equal(got, oracle.dijkstra(rp, ci, w, 0))


def test_int32_domain_wraps_like_numpy_int32():
    """The int32 domain (GraphBLAS C API, which the paper defers to):
    results are taken modulo 2^32.  Worked by hand, and against numpy's
    int32 arithmetic, which wraps the same way."""
    big = 2 ** 31 - 1
    A = S.Mat(1, 2, {(0, 0): big, (0, 1): 1}, "int32")
    ones = S.Mat(2, 1, {(0, 0): 1, (1, 0): 1}, "bool")
    C = S.mxm(S.Mat(1, 1, {}, "int32"), None, None, "plus.first", A, ones)
    assert C.e == {(0, 0): -2 ** 31}
    # the product is stored as int32 before the accumulator: min(5, -2^31)
    C = S.mxm(S.Mat(1, 1, {(0, 0): 5}, "int32"), None, "min", "plus.first", A, ones)
    assert C.e == {(0, 0): -2 ** 31}
    # an int64 output of the same product does not wrap
    A64 = S.Mat(1, 2, {(0, 0): big, (0, 1): 1}, "int64")
    assert S.mxm(S.Mat(1, 1, {}, "int64"), None, None, "plus.first", A64, ones).e == {(0, 0): 2 ** 31}
    X = S.Mat(1, 2, {(0, 0): 65536, (0, 1): 3}, "int32")
    Y = S.Mat(1, 2, {(0, 0): 65536, (0, 1): -7}, "int32")
    assert S.ewise_mult(S.Mat(1, 2, {}, "int32"), None, None, "times", X, Y).e == {(0, 0): 0, (0, 1): -21}
    rng = np.random.default_rng(5)
    vals = rng.integers(-2 ** 31, 2 ** 31, 40)
    M = S.Mat(5, 8, {(k // 8, k % 8): int(v) for k, v in enumerate(vals)}, "int32")
    assert S.reduce_scalar(M, "plus") == int(np.sum(vals.astype(np.int32), dtype=np.int32))
    w = S.reduce_rows(S.Vec(5, {}, "int32"), None, None, "plus", M)
    assert w.e == {i: int(np.sum(vals[8 * i:8 * i + 8].astype(np.int32), dtype=np.int32)) for i in range(5)}
    s = S.assign_scalar(S.Vec(3, {1: big}, "int32"), None, "plus", 1)
    assert s.e == {0: 1, 1: -2 ** 31, 2: 1}
