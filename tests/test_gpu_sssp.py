"""Parity of delta-stepping SSSP (Algorithm 5) on the device, through the C
ABI, with the oracle's Dijkstra.  Every distance is min over u of
fl(dist(u) + w(u, v)) with the final dist(u) on both sides, so the
comparison is bit for bit (integer weights make every sum exact; the
fractional case shows the same holds with rounding)."""
import math

import numpy as np
import pytest
import torch

import graphgen
import oracle
import graphs as Gs
from gpu_util import ctx, lagr

pytestmark = pytest.mark.gpu

DELTAS = (1.0, 8.0, 64.0, 300.0, 1e9)


def weighted_graph(rp, ci, w, directed=False):
    L = lagr()
    c = ctx()
    n = rp.size - 1
    A = L.Matrix.wrap_csr(c, n, n, torch.from_numpy(np.ascontiguousarray(rp)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(ci)).cuda(),
                          torch.from_numpy(np.ascontiguousarray(w, dtype=np.float64)).cuda())
    return L.Graph(c, A, L.ADJACENCY_DIRECTED if directed else L.ADJACENCY_UNDIRECTED)


def sssp(G, s, delta):
    L = lagr()
    return L.lagr_sssp(G, int(s), float(delta), ctx()).values_full(ctx()).cpu().numpy()


def rmat_weighted(scale, ef, seed, wseed, wmax=255):
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    rp, ci = oracle.build_adjacency(n, s, d)
    return n, s, d, rp, ci, graphgen.edge_weights(rp, ci, wseed, wmax)


def assert_same(got, want, label=""):
    assert got.dtype == np.float64 and got.shape == want.shape, label
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{label}: {bad.size} distances differ, first at {bad[:5]}: " \
                          f"{got[bad[:5]]} vs {want[bad[:5]]}"


@pytest.mark.parametrize("delta", DELTAS)
def test_rmat_s10_every_delta(delta):
    n, s, d, rp, ci, w = rmat_weighted(10, 16, 1, 5)
    G = weighted_graph(rp, ci, w)
    for src in graphgen.sources(n, s, d, 3, 7):
        assert_same(sssp(G, src, delta), oracle.dijkstra(rp, ci, w, int(src)), f"src {src} delta {delta}")


def test_rmat_s12_small_weights_many_ties():
    n, s, d, rp, ci, w = rmat_weighted(12, 8, 102, 9, wmax=4)
    G = weighted_graph(rp, ci, w)
    for src, delta in zip(graphgen.sources(n, s, d, 3, 11), (1.0, 2.0, 3.5)):
        assert_same(sssp(G, src, delta), oracle.dijkstra(rp, ci, w, int(src)), f"src {src}")


def test_fractional_weights_bit_exact():
    n, s, d, rp, ci, w = rmat_weighted(11, 16, 4, 6)
    w = w / 7.0 + 0.013
    G = weighted_graph(rp, ci, w)
    for src, delta in zip(graphgen.sources(n, s, d, 2, 12), (0.7, 5.0)):
        assert_same(sssp(G, src, delta), oracle.dijkstra(rp, ci, w, int(src)), f"src {src}")


def test_path_prefix_sums_and_grid():
    n, e = Gs.path(300)
    rp, ci = oracle.from_edges(n, e)
    w = graphgen.edge_weights(rp, ci, 3, 9)
    got = sssp(weighted_graph(rp, ci, w), 0, 4.0)
    # along a path the distance is the prefix sum of the edge weights
    steps = np.array([w[rp[i]:rp[i + 1]][ci[rp[i]:rp[i + 1]] == i + 1][0] for i in range(n - 1)])
    assert_same(got, np.concatenate([[0.0], np.cumsum(steps)]), "path")
    n, e = Gs.grid(23, 31)
    rp, ci = oracle.from_edges(n, e)
    got = sssp(weighted_graph(rp, ci, np.ones(ci.size)), 0, 1.0)
    r, c = np.divmod(np.arange(n), 31)
    assert_same(got, (r + c).astype(np.float64), "grid (Manhattan distance)")


def test_unreachable_isolated_and_single_vertex():
    n, e = Gs.disjoint_union(Gs.cycle(40), Gs.petersen())
    n += 3                                     # three isolated vertices
    rp, ci = oracle.from_edges(n, e)
    w = graphgen.edge_weights(rp, ci, 4, 30)
    G = weighted_graph(rp, ci, w)
    got = sssp(G, 5, 10.0)
    assert_same(got, oracle.dijkstra(rp, ci, w, 5), "two components")
    assert np.isinf(got[40:]).all() and np.isfinite(got[:40]).all()
    got = sssp(G, n - 1, 10.0)
    want = np.full(n, math.inf)
    want[n - 1] = 0.0
    assert_same(got, want, "isolated source")
    one = weighted_graph(np.zeros(2, np.int64), np.zeros(0, np.int32), np.zeros(0))
    assert_same(sssp(one, 0, 1.0), np.zeros(1), "one vertex")


def test_directed_graph_follows_out_edges():
    n, s, d = graphgen.rmat_edges(11, 8, 31)
    keep = s != d
    key = np.unique(s[keep].astype(np.int64) * n + d[keep])
    u, v = key // n, key % n
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, u + 1, 1)
    rp = np.cumsum(rp)
    ci = v.astype(np.int32)
    w = (np.arange(ci.size) * 2654435761 % 97 + 1).astype(np.float64)
    G = weighted_graph(rp, ci, w, directed=True)
    for src in graphgen.sources(n, s, d, 3, 13):
        assert_same(sssp(G, src, 16.0), oracle.dijkstra(rp, ci, w, int(src)), f"src {src}")


def test_alternating_graphs_reuse_the_context():
    a = rmat_weighted(9, 16, 41, 2)
    b = rmat_weighted(10, 4, 42, 3)
    Ga, Gb = weighted_graph(a[3], a[4], a[5]), weighted_graph(b[3], b[4], b[5])
    for _ in range(2):
        for (n, s, d, rp, ci, w), G in ((a, Ga), (b, Gb)):
            src = int(graphgen.sources(n, s, d, 1, 5)[0])
            assert_same(sssp(G, src, 32.0), oracle.dijkstra(rp, ci, w, src))


def test_full_size_rmat_s20():
    cfg = graphgen.LARGE
    n, s, d, rp, ci, w = rmat_weighted(cfg["scale"], cfg["edge_factor"], cfg["seed"], 20)
    G = weighted_graph(rp, ci, w)
    src = int(graphgen.sources(n, s, d, 1, 99)[0])
    assert_same(sssp(G, src, 32.0), oracle.dijkstra(rp, ci, w, src), "rmat s20")


def test_argument_errors():
    L = lagr()
    c = ctx()
    n, e = Gs.cycle(6)
    rp, ci = oracle.from_edges(n, e)
    G = weighted_graph(rp, ci, np.ones(ci.size))
    for bad in (0.0, -1.0, math.inf, math.nan):
        with pytest.raises(L.LagrError) as ex:
            L.lagr_sssp(G, 0, bad, c)
        assert ex.value.code == L.INVALID_VALUE
    for src in (-1, n):
        with pytest.raises(L.LagrError) as ex:
            L.lagr_sssp(G, src, 1.0, c)
        assert ex.value.code == L.INVALID_INDEX
    for bad in (0.0, -2.0, math.inf, math.nan):
        w = np.ones(ci.size)
        w[3] = bad
        with pytest.raises(L.LagrError) as ex:
            L.lagr_sssp(weighted_graph(rp, ci, w), 0, 1.0, c)
        assert ex.value.code == L.INVALID_VALUE
    pattern = L.Graph(c, L.Matrix.wrap_csr(c, n, n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()))
    with pytest.raises(L.LagrError) as ex:
        L.lagr_sssp(pattern, 0, 1.0, c)
    assert ex.value.code == L.DOMAIN_MISMATCH
