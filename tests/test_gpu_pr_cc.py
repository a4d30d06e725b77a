"""PageRank (Algorithm 4) and FastSV connected components (Algorithm 7) on
the device, through the C ABI, against the oracle.

PageRank tolerance: an iteration adds, for every vertex, k non-negative
terms; the device adds a row of at most 32 in-edges in the listing's
ascending order (the same bits) and longer rows in another fixed order,
which changes the sum by at most (k - 1) * 2^-53 relative.  With no row
longer than 32 every iteration gives the oracle's bits from the oracle's
inputs, so the ranks are equal.  Otherwise let kmax (> 32) be the most
in-edges of a vertex.  An iteration's new rank is the exact teleport term
plus damping a times a weighted sum of the old ranks with non-negative
weights, so a relative error E in every old rank gives at most a * E in
the new one, plus the two roundings of at most kmax - 1 additions each:
after T iterations the relative error is at most 4 * kmax * 2^-53 * (1 +
a + ... + a^(T-1)) (the factor 4 also covers the teleport add and the
divisions).  The observed largest error is checked
to lie under that bound and is shown beside it when it does not.  The
iteration count must match exactly.  Components are integer labels:
bit-exact."""
import math

import numpy as np
import pytest
import torch

import graphgen
import oracle
import graphs as Gs
from gpu_util import ctx, lagr

pytestmark = pytest.mark.gpu


def graph_of(rp, ci, directed=False):
    L = lagr()
    c = ctx()
    n = rp.size - 1
    A = L.Matrix.wrap_csr(c, n, n, torch.from_numpy(np.ascontiguousarray(rp)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(ci)).cuda())
    return L.Graph(c, A, L.ADJACENCY_DIRECTED if directed else L.ADJACENCY_UNDIRECTED)


def rmat_graph(scale, ef, seed, directed=False):
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    rp, ci = (oracle.build_directed if directed else oracle.build_adjacency)(n, s, d)
    return rp, ci, graph_of(rp, ci, directed)


def pagerank(G, damping=0.85, tol=1e-4, itermax=100):
    L = lagr()
    v, k = L.lagr_pagerank(G, ctx(), damping, tol, itermax)
    return v.values_full(ctx()).cpu().numpy(), k


def rank_bound(iters, rp, ci, damping=0.85):
    indeg = np.bincount(ci, minlength=rp.size - 1) if ci.size else np.zeros(1, dtype=np.int64)
    long_rows = indeg[indeg > 32]
    if long_rows.size == 0:
        return 0.0
    return 4.0 * float(long_rows.max()) * 2.0 ** -53 * sum(damping ** t for t in range(max(iters, 1)))


def assert_rank_close(got, want, iters, rp, ci):
    rtol = rank_bound(iters, rp, ci)
    err = np.abs(got - want) / np.abs(want)
    assert err.max() <= rtol, f"max rel err {err.max():.3e} > bound {rtol:.3e}"
    return float(err.max()), rtol


@pytest.mark.parametrize("scale,ef,seed,directed", [(10, 16, 301, False), (12, 8, 302, False),
                                                    (11, 16, 303, True)])
def test_pagerank_matches_the_oracle(scale, ef, seed, directed):
    rp, ci, G = rmat_graph(scale, ef, seed, directed)
    for tol, itermax in ((0.0, 20), (1e-4, 100), (1e-9, 200)):
        got, k = pagerank(G, 0.85, tol, itermax)
        want, ko = oracle.pagerank(rp, ci, 0.85, tol, itermax)
        assert k == ko, (tol, k, ko)
        err, bound = assert_rank_close(got, want, k, rp, ci)
        print(f"\npagerank s{scale}: {k} iterations, largest relative error {err:.3e}, bound {bound:.3e}")
    # a second run gives the same bits
    again, _ = pagerank(G, 0.85, 1e-9, 200)
    assert np.array_equal(again, pagerank(G, 0.85, 1e-9, 200)[0])


def test_pagerank_short_rows_are_bit_exact():
    """Every in-degree <= 32: the device adds in the listing's order."""
    n, e = Gs.grid(17, 23)
    rp, ci = oracle.from_edges(n, e)
    got, k = pagerank(graph_of(rp, ci), 0.85, 1e-10, 300)
    want, ko = oracle.pagerank(rp, ci, 0.85, 1e-10, 300)
    assert k == ko and np.array_equal(got, want)


def test_pagerank_closed_forms_and_edges():
    L = lagr()
    a = 0.85
    n, e = Gs.complete(40)
    rp, ci = oracle.from_edges(n, e)
    got, k = pagerank(graph_of(rp, ci), a, 1e-12, 100)
    assert k == 1 and np.allclose(got, 1.0 / n, rtol=1e-14, atol=0)
    n, e = Gs.star(70)
    rp, ci = oracle.from_edges(n, e)
    got, _ = pagerank(graph_of(rp, ci), a, 1e-15, 2000)
    b = (1 - a) / n
    rc = b * (1 + (n - 1) * a) / (1 - a * a)
    assert np.allclose(got, [rc] + [b + a * rc / (n - 1)] * (n - 1), rtol=1e-12, atol=0)
    rp, ci, G = rmat_graph(9, 8, 304)
    got, k = pagerank(G, a, 1e-4, 0)
    assert k == 0 and np.all(got == 1.0 / (rp.size - 1))
    for damping, tol, itermax in ((-0.1, 1e-4, 10), (1.5, 1e-4, 10), (math.nan, 1e-4, 10),
                                  (0.85, -1.0, 10), (0.85, math.inf, 10), (0.85, 1e-4, -1)):
        with pytest.raises(L.LagrError) as ex:
            L.lagr_pagerank(G, ctx(), damping, tol, itermax)
        assert ex.value.code == L.INVALID_VALUE


def test_pagerank_full_size_rmat_s20():
    cfg = graphgen.LARGE
    rp, ci, G = rmat_graph(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    got, k = pagerank(G, 0.85, 1e-4, 20)
    want, ko = oracle.pagerank(rp, ci, 0.85, 1e-4, 20)
    assert k == ko
    err, bound = assert_rank_close(got, want, k, rp, ci)
    print(f"\npagerank 2^20: {k} iterations, largest relative error {err:.3e}, bound {bound:.3e}")


@pytest.mark.parametrize("scale,ef,seed,directed", [(10, 2, 311, False), (14, 2, 312, False),
                                                    (12, 1, 313, True), (13, 16, 314, False)])
def test_components_match_the_oracle(scale, ef, seed, directed):
    L = lagr()
    rp, ci, G = rmat_graph(scale, ef, seed, directed)
    lab, iters = L.lagr_cc(G, ctx())
    got = lab.values_full(ctx()).cpu().numpy()
    assert np.array_equal(got, oracle.components(rp, ci, directed=directed)) and iters >= 1


def test_components_closed_forms_and_full_size():
    L = lagr()
    n, e = Gs.disjoint_union(Gs.path(300), Gs.disjoint_union(Gs.petersen(), Gs.star(1000)))
    rp, ci = oracle.from_edges(n + 5, e)                      # five isolated vertices
    got = L.lagr_cc(graph_of(rp, ci), ctx())[0].values_full(ctx()).cpu().numpy()
    want = np.array([0] * 300 + [300] * 10 + [310] * 1000 + list(range(1310, 1315)))
    assert np.array_equal(got, want)
    empty = graph_of(np.zeros(8, np.int64), np.zeros(0, np.int32))
    assert np.array_equal(L.lagr_cc(empty, ctx())[0].values_full(ctx()).cpu().numpy(), np.arange(7))
    cfg = graphgen.LARGE
    rp, ci, G = rmat_graph(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    got = L.lagr_cc(G, ctx())[0].values_full(ctx()).cpu().numpy()
    assert np.array_equal(got, oracle.components(rp, ci))
