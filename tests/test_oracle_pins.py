"""Pins of the CPU oracle against facts fixed by the paper and by
mathematics: closed forms, invariants, brute force and independent
libraries.  None of these re-types the oracle's own code."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import oracle
import graphs as G


def adj(g):
    n, e = g
    return oracle.from_edges(n, e)


def brute_triangles(A):
    n = A.shape[0]
    return sum(1 for i, j, k in itertools.combinations(range(n), 3)
               if A[i, j] and A[j, k] and A[i, k])


# ---------------------------------------------------------------- TC (Alg 6)

@pytest.mark.parametrize("n", range(3, 13))
def test_tc_complete_graph(n):
    assert oracle.triangle_count(*adj(G.complete(n))) == math.comb(n, 3)


@pytest.mark.parametrize("g", [G.path(9), G.cycle(4), G.cycle(7), G.star(8),
                               G.complete_bipartite(3, 5), G.petersen(), G.grid(4, 5)])
def test_tc_triangle_free(g):
    assert oracle.triangle_count(*adj(g)) == 0


def test_tc_random_trees_are_triangle_free():
    rng = np.random.default_rng(7)
    for n in (2, 5, 30, 100):
        assert oracle.triangle_count(*adj(G.random_tree(n, rng))) == 0


@pytest.mark.parametrize("m", range(4, 12))
def test_tc_wheel(m):
    assert oracle.triangle_count(*adj(G.wheel(m))) == m


def test_tc_triangle_and_wheel3():
    assert oracle.triangle_count(*adj(G.cycle(3))) == 1
    # W_3 is K_4
    assert oracle.triangle_count(*adj(G.wheel(3))) == 4


def test_tc_disjoint_union_adds():
    g = G.disjoint_union(G.complete(6), G.wheel(7))
    assert oracle.triangle_count(*adj(g)) == 20 + 7


def test_tc_trace_and_brute_force_and_relabel():
    rng = np.random.default_rng(11)
    for n, p in [(12, 0.5), (30, 0.3), (60, 0.15), (64, 0.4)]:
        g = G.random_graph(n, p, rng)
        A = G.dense(g)
        t = oracle.triangle_count(*adj(g))
        assert t == int(np.trace(A @ A @ A)) // 6
        if n <= 30:
            assert t == brute_triangles(A)
        perm = rng.permutation(n)
        assert oracle.triangle_count(*adj(G.relabel(g, perm))) == t


def test_tc_lower_counts_match_masked_integer_product():
    """C<s(L)> = L plus.pair L' is, on 0/1 patterns, the integer product
    L @ L' restricted to L's pattern; its sum is the triangle count."""
    rng = np.random.default_rng(5)
    for n, p in [(20, 0.4), (50, 0.2), (64, 0.5)]:
        g = G.random_graph(n, p, rng)
        A = G.dense(g)
        L = np.tril(A, -1)
        P = L @ L.T
        lrp, lci, cnt = oracle.lower_counts(*adj(g))
        rows = np.repeat(np.arange(n), np.diff(lrp))
        assert np.array_equal(L[rows, lci], np.ones_like(lci))
        assert lci.size == int(L.sum())
        assert np.array_equal(cnt, P[rows, lci])
        assert int(cnt.sum()) == oracle.triangle_count(*adj(g))


def test_tc_rows_partition_sums_to_total():
    rng = np.random.default_rng(3)
    g = G.random_graph(80, 0.2, rng)
    rp, ci = adj(g)
    parts = sum(oracle.triangle_count_rows(rp, ci, a, a + 17) for a in range(0, 80, 17))
    assert parts == oracle.triangle_count(rp, ci)
    strided = sum(oracle.triangle_count_rows(rp, ci, r, 80, 3) for r in range(3))
    assert strided == oracle.triangle_count(rp, ci)


# ------------------------------------------------------------- BFS (Alg 1/2)

def check_parent_tree(rp, ci, s, level, parent):
    n = rp.size - 1
    nb = [set(ci[rp[v]:rp[v + 1]].tolist()) for v in range(n)]
    assert parent[s] == s and level[s] == 0
    for v in range(n):
        if level[v] < 0:
            assert parent[v] == -1
        elif v != s:
            p = parent[v]
            assert p in nb[v] and level[p] == level[v] - 1


def test_bfs_path_star_grid():
    rp, ci = adj(G.path(10))
    lv, pa = oracle.bfs(rp, ci, 0)
    assert lv.tolist() == list(range(10))
    assert pa.tolist() == [0] + list(range(9))
    rp, ci = adj(G.star(9))
    lv, _ = oracle.bfs(rp, ci, 0)
    assert lv.tolist() == [0] + [1] * 8
    lv, _ = oracle.bfs(rp, ci, 3)
    assert lv.tolist() == [1, 2, 2, 0, 2, 2, 2, 2, 2]
    r, c = 5, 7
    rp, ci = adj(G.grid(r, c))
    lv, pa = oracle.bfs(rp, ci, 0)
    assert lv.tolist() == [i + j for i in range(r) for j in range(c)]
    check_parent_tree(rp, ci, 0, lv, pa)


def test_bfs_levels_are_shortest_distances():
    rng = np.random.default_rng(2)
    for n, p in [(40, 0.05), (70, 0.03), (64, 0.1)]:
        g = G.random_graph(n, p, rng)
        rp, ci = adj(g)
        A = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
        D = csg.shortest_path(A, unweighted=True, directed=False)
        for s in (0, n // 2, n - 1):
            lv, pa = oracle.bfs(rp, ci, s)
            want = np.where(np.isinf(D[s]), -1, D[s]).astype(np.int64)
            assert np.array_equal(lv.astype(np.int64), want)
            check_parent_tree(rp, ci, s, lv, pa)
            mp = oracle.bfs_min_parent(rp, ci, s, lv)
            check_parent_tree(rp, ci, s, lv, mp)
            for v in range(n):
                if lv[v] > 0:
                    cands = [u for u in ci[rp[v]:rp[v + 1]] if lv[u] == lv[v] - 1]
                    assert mp[v] == min(cands)


def test_bfs_reached_set_is_component():
    g = G.disjoint_union(G.cycle(6), G.path(4))
    rp, ci = adj(g)
    lv, pa = oracle.bfs(rp, ci, 7)
    assert (lv[:6] == -1).all() and (pa[:6] == -1).all()
    assert lv[6:].tolist() == [1, 0, 1, 2]


# -------------------------------------------------------------- BC (Alg 3)

def brute_bc(A, sources):
    """Sum over s in sources, t != s, of the fraction of shortest s-t paths
    through v, by explicit enumeration of every shortest path."""
    n = A.shape[0]
    nb = [list(np.nonzero(A[v])[0]) for v in range(n)]
    out = np.zeros(n)
    for s in sources:
        dist = {s: 0}
        frontier = [s]
        while frontier:
            nxt = []
            for u in frontier:
                for w in nb[u]:
                    if w not in dist:
                        dist[w] = dist[u] + 1
                        nxt.append(w)
            frontier = nxt
        for t in dist:
            if t == s:
                continue
            paths = []

            def walk(p):
                if p[-1] == t:
                    paths.append(p)
                    return
                for w in nb[p[-1]]:
                    if dist.get(w) == dist[p[-1]] + 1 and dist[w] <= dist[t]:
                        walk(p + [w])

            walk([s])
            for p in paths:
                for v in p[1:-1]:
                    out[v] += 1.0 / len(paths)
    return out


def test_bc_path_all_sources():
    n = 9
    rp, ci = adj(G.path(n))
    got = oracle.brandes(rp, ci, np.arange(n))
    assert np.allclose(got, [2 * i * (n - 1 - i) for i in range(n)], rtol=0, atol=1e-12)


def test_bc_path_single_source():
    n = 7
    rp, ci = adj(G.path(n))
    got = oracle.brandes(rp, ci, [0])
    assert got.tolist() == [0.0] + [float(n - 1 - i) for i in range(1, n)]


def test_bc_star_complete_cycle():
    n = 8
    rp, ci = adj(G.star(n))
    got = oracle.brandes(rp, ci, np.arange(n))
    assert got[0] == (n - 1) * (n - 2) and (got[1:] == 0).all()
    rp, ci = adj(G.complete(7))
    assert (oracle.brandes(rp, ci, np.arange(7)) == 0).all()
    rp, ci = adj(G.cycle(9))
    got = oracle.brandes(rp, ci, np.arange(9))
    assert np.allclose(got, got[0]) and got[0] > 0


def test_bc_sum_invariant_and_brute_force():
    rng = np.random.default_rng(13)
    for n, p in [(9, 0.35), (10, 0.3), (12, 0.25)]:
        g = G.random_graph(n, p, rng)
        A = G.dense(g)
        rp, ci = adj(g)
        S = rng.choice(n, size=4, replace=False)
        got = oracle.brandes(rp, ci, S)
        assert np.allclose(got, brute_bc(A, S), rtol=1e-12, atol=1e-12)
        # sum over v of BC(v) = sum over s, reached t != s, of d(s,t) - 1
        tot = 0
        for s in S:
            lv, _ = oracle.bfs(rp, ci, int(s))
            tot += int(np.sum(lv[lv > 0] - 1))
        assert abs(got.sum() - tot) <= 1e-9 * max(1, tot)


def test_bc_against_networkx_subset():
    nx = pytest.importorskip("networkx")
    rng = np.random.default_rng(17)
    n, e = G.random_graph(60, 0.08, rng)
    rp, ci = oracle.from_edges(n, e)
    S = [int(x) for x in rng.choice(n, size=8, replace=False)]
    Gx = nx.Graph()
    Gx.add_nodes_from(range(n))
    Gx.add_edges_from(e)
    ref = nx.betweenness_centrality_subset(Gx, S, list(range(n)), normalized=False)
    got = oracle.brandes(rp, ci, S)
    # networkx halves undirected pair counts; the paper's sum does not
    assert np.allclose(got, [2 * ref[v] for v in range(n)], rtol=1e-12, atol=1e-12)


# ------------------------------------------------------ graph construction

def test_build_symmetric_sorted_unique_no_loops():
    import graphgen
    n, s, d = graphgen.rmat_edges(8, 8, 123)
    rp, ci = oracle.build_adjacency(n, s, d)
    A = sp.csr_matrix((np.ones(s.size), (s, d)), shape=(n, n)).toarray() != 0
    A = (A | A.T)
    np.fill_diagonal(A, False)
    B = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n)).toarray() != 0
    assert (A == B).all()
    for v in range(n):
        row = ci[rp[v]:rp[v + 1]]
        assert (np.diff(row) > 0).all() and v not in row


# ------------------------------------------------------------- SSSP (Alg 5)

def weighted(n, edges, seed=7, wmax=255):
    import graphgen
    rp, ci = oracle.from_edges(n, edges)
    return rp, ci, graphgen.edge_weights(rp, ci, seed, wmax)


def test_edge_weights_are_symmetric_integers():
    import graphgen
    n, s, d = graphgen.rmat_edges(9, 8, 12)
    rp, ci = oracle.build_adjacency(n, s, d)
    w = graphgen.edge_weights(rp, ci, 3)
    M = sp.csr_matrix((w, ci, rp), shape=(n, n))
    assert (M != M.T).nnz == 0
    assert w.min() >= 1 and w.max() <= 255 and np.array_equal(w, np.round(w))


def test_sssp_unit_weights_are_bfs_levels():
    import graphgen
    n, s, d = graphgen.rmat_edges(10, 16, 1)
    rp, ci = oracle.build_adjacency(n, s, d)
    src = int(graphgen.sources(n, s, d, 1, 1)[0])
    dist = oracle.dijkstra(rp, ci, np.ones(ci.size), src)
    lev = oracle.bfs(rp, ci, src)[0]
    assert np.array_equal(np.where(lev >= 0, lev.astype(float), np.inf), dist)


def test_sssp_path_prefix_sums_and_grid():
    n = 40
    rp, ci, w = weighted(*G.path(n))
    dist = oracle.dijkstra(rp, ci, w, 0)
    step = [w[rp[i]:rp[i + 1]][ci[rp[i]:rp[i + 1]] == i + 1][0] for i in range(n - 1)]
    assert np.array_equal(dist, np.concatenate([[0.0], np.cumsum(step)]))
    rp, ci = adj(G.grid(7, 9))
    dist = oracle.dijkstra(rp, ci, np.ones(ci.size), 0)
    assert np.array_equal(dist, np.array([i + j for i in range(7) for j in range(9)], dtype=float))


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sssp_against_scipy_and_floyd_warshall(seed):
    rng = np.random.default_rng(seed)
    n = 24
    rp, ci, w = weighted(*G.random_graph(n, 0.15, rng), seed=seed)
    M = sp.csr_matrix((w, ci, rp), shape=(n, n))
    FW = csg.floyd_warshall(M, directed=True)
    # textbook Floyd-Warshall by hand as well (integer weights: every sum exact)
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    for u in range(n):
        for p in range(rp[u], rp[u + 1]):
            D[u, ci[p]] = min(D[u, ci[p]], w[p])
    for k in range(n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    assert np.array_equal(D, FW)
    for s in range(n):
        assert np.array_equal(oracle.dijkstra(rp, ci, w, s), D[s])


def test_sssp_rmat_against_scipy_dijkstra():
    import graphgen
    n, s, d = graphgen.rmat_edges(11, 8, 21)
    rp, ci = oracle.build_adjacency(n, s, d)
    w = graphgen.edge_weights(rp, ci, 21)
    M = sp.csr_matrix((w, ci, rp), shape=(n, n))
    for src in graphgen.sources(n, s, d, 4, 21):
        want = csg.dijkstra(M, directed=True, indices=int(src))
        assert np.array_equal(oracle.dijkstra(rp, ci, w, int(src)), want)
