"""Pins of the CPU oracle against facts fixed by the paper and by
mathematics: closed forms, invariants, brute force and independent
libraries.  None of these re-types the oracle's own code."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

import graphgen
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


# ------------------------------------------------------ directed graphs
# A(u, v) is the edge u -> v (Section II, LAGRAPH_ADJACENCY_DIRECTED); pull
# steps and the BC predecessor sweep read in-edges, the rows of AT.

def _digraph(scale, ef, seed):
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    rp, ci = oracle.build_directed(n, s, d)
    return n, s, d, rp, ci


def _dense(n, rp, ci, vals=None):
    M = np.zeros((n, n))
    for u in range(n):
        M[u, ci[rp[u]:rp[u + 1]]] = 1.0 if vals is None else vals[rp[u]:rp[u + 1]]
    return M


def test_build_directed_is_the_set_of_draws():
    n, s, d = graphgen.rmat_edges(8, 8, 61)
    rp, ci = oracle.build_directed(n, s, d)
    want = sorted(set((int(a), int(b)) for a, b in zip(s, d) if a != b))
    got = [(u, int(v)) for u in range(n) for v in ci[rp[u]:rp[u + 1]]]
    assert got == want


def test_transpose_is_the_dense_transpose():
    for seed in (71, 72, 73):
        n, _, _, rp, ci = _digraph(7, 6, seed)
        w = np.arange(1, ci.size + 1, dtype=np.float64)
        rpT, ciT, wT = oracle.transpose(rp, ci, values=w)
        assert np.array_equal(_dense(n, rpT, ciT, wT), _dense(n, rp, ci, w).T)
        assert all(np.all(np.diff(ciT[rpT[u]:rpT[u + 1]]) > 0) for u in range(n))
        r2, c2 = oracle.transpose(rpT, ciT)
        assert np.array_equal(r2, rp) and np.array_equal(c2, ci)
    rpT, ciT = oracle.transpose(np.array([0, 2, 3]), np.array([1, 4, 0], np.int32), ncols=5)
    assert rpT.tolist() == [0, 1, 2, 2, 2, 3] and ciT.tolist() == [1, 0, 0]


def test_directed_bfs_levels_and_in_neighbour_parents():
    n, s, d, rp, ci = _digraph(7, 8, 75)
    D = _dense(n, rp, ci) > 0
    rpT, ciT = oracle.transpose(rp, ci)
    for src in graphgen.sources(n, s, d, 4, 3):
        src = int(src)
        level, _ = oracle.bfs(rp, ci, src)
        # levels: first k with v in the k-step reach set (boolean powers of A)
        want = np.full(n, -1)
        reach = np.zeros(n, bool)
        reach[src] = True
        want[src] = 0
        k = 0
        while True:
            k += 1
            nxt = (reach[:, None] & D).any(axis=0) & ~reach
            if not nxt.any():
                break
            want[nxt] = k
            reach |= nxt
        assert np.array_equal(level, want)
        par = oracle.bfs_min_parent(rpT, ciT, src, level)
        assert par[src] == src
        for v in range(n):
            if v == src:
                continue
            cands = [u for u in range(n) if D[u, v] and level[v] > 0 and level[u] == level[v] - 1]
            assert par[v] == (min(cands) if cands else -1), v


def _bc_by_definition(n, rp, ci, sources):
    """Sum over s in sources, t != s, v not in {s, t} of sigma_st(v) /
    sigma_st, from exact all-pairs shortest-path counts."""
    from fractions import Fraction
    dist = [[-1] * n for _ in range(n)]
    sig = [[0] * n for _ in range(n)]
    for a in range(n):
        dist[a][a], sig[a][a] = 0, 1
        frontier = [a]
        while frontier:
            nxt = []
            for u in frontier:
                for v in ci[rp[u]:rp[u + 1]]:
                    v = int(v)
                    if dist[a][v] < 0:
                        dist[a][v] = dist[a][u] + 1
                        nxt.append(v)
                    if dist[a][v] == dist[a][u] + 1:
                        sig[a][v] += sig[a][u]
            frontier = nxt
    bc = [Fraction(0)] * n
    for s_ in sources:
        for t in range(n):
            if t == s_ or dist[s_][t] < 0:
                continue
            for v in range(n):
                if v in (s_, t) or dist[s_][v] < 0 or dist[v][t] < 0:
                    continue
                if dist[s_][v] + dist[v][t] == dist[s_][t]:
                    bc[v] += Fraction(sig[s_][v] * sig[v][t], sig[s_][t])
    return np.array([float(x) for x in bc])


@pytest.mark.parametrize("scale,ef,seed", [(4, 6, 81), (5, 4, 82), (5, 8, 83)])
def test_brandes_directed_matches_the_definition(scale, ef, seed):
    n, _, _, rp, ci = _digraph(scale, ef, seed)
    srcs = np.arange(n)
    got = oracle.brandes_directed(rp, ci, srcs)
    want = _bc_by_definition(n, rp, ci, srcs)
    assert np.allclose(got, want, rtol=1e-12, atol=0) and np.array_equal(got == 0, want == 0)


def test_brandes_directed_closed_forms_and_symmetric_case():
    n = 9
    rp, ci = oracle.build_directed(n, np.arange(n - 1), np.arange(1, n))       # path 0 -> ... -> 8
    k = np.arange(n)
    assert np.array_equal(oracle.brandes_directed(rp, ci, k), (k * (n - 1 - k)).astype(np.float64))
    rp, ci = oracle.build_directed(n, np.arange(n), (np.arange(n) + 1) % n)    # directed cycle
    assert np.array_equal(oracle.brandes_directed(rp, ci, k), np.full(n, (n - 1) * (n - 2) / 2))
    n, s, d = graphgen.rmat_edges(8, 8, 84)
    rp, ci = oracle.build_adjacency(n, s, d)                                  # symmetric: A = AT
    srcs = graphgen.sources(n, s, d, 16, 5)
    assert np.allclose(oracle.brandes_directed(rp, ci, srcs), oracle.brandes(rp, ci, srcs), rtol=1e-12, atol=0)


# ------------------------------------------------------------- PageRank
# Algorithm 4 (GAP): r <- (1 - a)/n + a * AT D+ r, where D+ = diag(1/d_out)
# on vertices with out-edges and 0 on the others (they send nothing).

def _pagerank_dense(rp, ci, damping, iters):
    n = rp.size - 1
    A = _dense(n, rp, ci)
    dout = A.sum(axis=1)
    dplus = np.where(dout > 0, 1.0 / np.where(dout > 0, dout, 1.0), 0.0)
    r = np.full(n, 1.0 / n)
    hist = []
    for _ in range(iters):
        t = r
        r = (1.0 - damping) / n + damping * (A.T @ (dplus * t))
        hist.append(np.abs(t - r).sum())
    return r, hist


@pytest.mark.parametrize("directed,seed", [(False, 91), (True, 92), (False, 93)])
def test_pagerank_is_the_dense_power_iteration(directed, seed):
    n, s, d = graphgen.rmat_edges(7, 6, seed)
    rp, ci = (oracle.build_directed if directed else oracle.build_adjacency)(n, s, d)
    for iters in (1, 2, 7, 30):
        got, k = oracle.pagerank(rp, ci, 0.85, 0.0, iters)
        want, _ = _pagerank_dense(rp, ci, 0.85, iters)
        assert k == iters
        assert np.allclose(got, want, rtol=1e-12, atol=0)
    # the stopping rule: the first iteration whose change has 1-norm < tol
    _, hist = _pagerank_dense(rp, ci, 0.85, 100)
    for tol in (1e-2, 1e-4, 1e-7):
        first = next(i + 1 for i, h in enumerate(hist) if h < tol)
        if min(abs(h - tol) for h in hist) > 1e-9 * tol:
            assert oracle.pagerank(rp, ci, 0.85, tol, 100)[1] == first


def test_pagerank_closed_forms():
    a = 0.85
    for n, e in (G.complete(12), G.cycle(10)):
        rp, ci = oracle.from_edges(n, e)
        r, k = oracle.pagerank(rp, ci, a, 1e-12, 100)
        assert np.allclose(r, 1.0 / n, rtol=1e-14, atol=0) and k == 1
    rp, ci = oracle.build_directed(7, np.arange(7), (np.arange(7) + 1) % 7)    # directed cycle
    r, _ = oracle.pagerank(rp, ci, a, 1e-12, 100)
    assert np.allclose(r, 1.0 / 7, rtol=1e-14, atol=0)
    n, e = G.star(9)                                  # centre 0, eight leaves
    rp, ci = oracle.from_edges(n, e)
    r, _ = oracle.pagerank(rp, ci, a, 1e-15, 1000)
    b = (1 - a) / n
    rc = b * (1 + (n - 1) * a) / (1 - a * a)
    rl = b + a * rc / (n - 1)
    assert np.allclose(r, [rc] + [rl] * (n - 1), rtol=1e-12, atol=0)
    assert abs(rc + (n - 1) * rl - 1.0) < 1e-12
    # an isolated vertex keeps only the teleport share and sends nothing
    rp, ci = oracle.from_edges(4, [(0, 1), (1, 2)])
    r, _ = oracle.pagerank(rp, ci, a, 1e-14, 1000)
    assert r[3] == (1 - a) / 4 and r.sum() < 1.0


# ---------------------------------------------------- connected components

@pytest.mark.parametrize("directed,seed", [(False, 95), (True, 96), (False, 97)])
def test_components_are_min_ids_of_scipy_components(directed, seed):
    n, s, d = graphgen.rmat_edges(11, 2, seed)
    rp, ci = (oracle.build_directed if directed else oracle.build_adjacency)(n, s, d)
    lab = oracle.components(rp, ci, directed=directed)
    M = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    k, comp = csg.connected_components(M, directed=directed, connection="weak")
    assert len(set(lab.tolist())) == k > 1
    for c in range(k):
        members = np.nonzero(comp == c)[0]
        assert (lab[members] == members.min()).all()


def test_components_closed_forms():
    n, e = G.disjoint_union(G.path(5), G.disjoint_union(G.petersen(), G.star(4)))
    rp, ci = oracle.from_edges(n + 2, e)              # two isolated vertices at the end
    want = [0] * 5 + [5] * 10 + [15] * 4 + [19, 20]
    assert oracle.components(rp, ci).tolist() == want
    rp, ci = oracle.build_directed(4, np.array([3, 2, 1]), np.array([2, 1, 0]))   # 3 -> 2 -> 1 -> 0
    assert oracle.components(rp, ci, directed=True).tolist() == [0, 0, 0, 0]
