"""Parity of the device path (through the C ABI) with the CPU oracle:
graph build, triangle counting, BFS and betweenness centrality."""
import json
import math
import os

import numpy as np
import pytest
import torch

import graphgen
import oracle
import graphs as Gs
from gpu_util import (assert_bc_close, check_parents, ctx, device_graph, graph_csr,
                      graph_from_edges, lagr, rmat)

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_values.json")))


# --------------------------------------------------------------- build

@pytest.mark.parametrize("scale,ef,seed", [(8, 4, 101), (10, 16, 1), (12, 8, 102)])
def test_device_build_equals_oracle_adjacency(scale, ef, seed):
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    rp, ci = graph_csr(G)
    orp, oci = oracle.build_adjacency(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)


def test_build_empty_and_all_loops():
    G, (orp, oci) = graph_from_edges(5, [(1, 1), (3, 3)])
    rp, ci = graph_csr(G)
    assert rp.tolist() == [0] * 6 and ci.size == 0
    L = lagr()
    assert L.lagr_tc(G, ctx()) == 0


def test_graph_check_rejects_malformed():
    import torch
    L = lagr()
    c = ctx()
    cases = {
        "unsorted": ([0, 2, 3, 4], [2, 1, 0, 0]),
        "duplicate": ([0, 2, 3, 4], [1, 1, 0, 0]),
        "asymmetric": ([0, 1, 1, 1], [1]),
        "out of range": ([0, 1, 2, 2], [5, 0]),
    }
    for name, (rp, ci) in cases.items():
        rpt = torch.tensor(rp, dtype=torch.int64, device="cuda")
        cit = torch.tensor(ci, dtype=torch.int32, device="cuda")
        A = L.Matrix.wrap_csr(c, 3, 3, rpt, cit)
        G = L.Graph(c, A)
        with pytest.raises(L.LagrError) as e:
            G.check(c)
        assert e.value.code == L.INVALID_OBJECT, name


# ------------------------------------------------------------------ TC

@pytest.mark.parametrize("n", [3, 4, 7, 16, 40, 90])
def test_tc_complete(n):
    G, _ = graph_from_edges(*Gs.complete(n))
    assert lagr().lagr_tc(G, ctx()) == math.comb(n, 3)


@pytest.mark.parametrize("g,want", [(Gs.wheel(5), 5), (Gs.wheel(30), 30), (Gs.petersen(), 0),
                                    (Gs.grid(6, 9), 0), (Gs.complete_bipartite(7, 9), 0),
                                    (Gs.disjoint_union(Gs.complete(9), Gs.wheel(11)), 84 + 11)])
def test_tc_closed_forms(g, want):
    G, _ = graph_from_edges(*g)
    assert lagr().lagr_tc(G, ctx()) == want


def test_tc_hub_rows_longer_than_the_lds_table():
    # a complete graph of 1500 vertices: rows of L reach 1499 > 1024 entries
    n = 1500
    G, _ = graph_from_edges(*Gs.complete(n))
    assert lagr().lagr_tc(G, ctx()) == math.comb(n, 3)


def test_tc_rows_longer_than_the_sort_tile():
    # K_2100: rows of L reach 2099 entries, past the LDS row sort (2048), so
    # L is sorted by the global radix sort instead
    n = 2100
    G, _ = graph_from_edges(*Gs.complete(n))
    assert lagr().lagr_tc(G, ctx()) == math.comb(n, 3)
    lrp, lci = lower_csr(G)
    assert lrp[-1] == n * (n - 1) // 2
    for r in (0, 1, 1000, n - 1):
        assert np.array_equal(lci[lrp[r]:lrp[r + 1]], np.arange(r))


def lower_csr(G):
    """(rowptr, colidx) of the graph's cached strictly lower part, on the host."""
    rp, ci, _ = G.tc_lower().to_csr(ctx())
    return rp.cpu().numpy(), ci.cpu().numpy()


def expected_lower(n, s, d):
    """(rowptr, colidx) of the strict lower part of A after relabelling by
    descending degree (ties by id), rows sorted, rebuilt with numpy from the
    oracle's adjacency."""
    rp, ci = oracle.build_adjacency(n, s, d)
    deg = np.diff(rp)
    order = np.lexsort((np.arange(n), -deg))
    inv = np.empty(n, dtype=np.int64)
    inv[order] = np.arange(n)
    rows = np.repeat(np.arange(n), deg)
    ni, nj = inv[rows], inv[ci]
    keep = nj < ni
    key = np.sort(ni[keep] * n + nj[keep])
    return np.searchsorted(key // n, np.arange(n + 1), side="left"), key % n


@pytest.mark.parametrize("scale,ef,seed", [(10, 16, 1), (11, 8, 5), (9, 32, 6)])
def test_tc_lower_is_the_degree_relabelled_lower_part(scale, ef, seed):
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    lagr().lagr_property_tc_lower(G, ctx())
    lrp, lci = lower_csr(G)
    want_rp, want_ci = expected_lower(n, s, d)
    assert np.array_equal(lrp, want_rp)
    assert np.array_equal(lci, want_ci)


def test_tc_lower_rows_of_every_sort_size():
    """A dense random graph with uneven edge probabilities (p(u,v) = w_u w_v,
    w near 1 for a core of 1,300 vertices): after the relabel, rows of L
    run from empty to over 1,024 ids in an order unrelated to the
    relabelled ids, so every size class of the row sort (rank sort up to 64
    ids, wave sorts of 2 to 32 chunks of 64) has rows to put in order.  L
    is compared with the numpy rebuild and the count with trace(A^3)/6."""
    rng = np.random.default_rng(77)
    n = 1400
    w = np.where(np.arange(n) % 14 == 0, rng.uniform(0.05, 0.5, n), rng.uniform(0.9, 1.0, n))
    iu, ju = np.triu_indices(n, 1)
    keep = rng.random(iu.size) < w[iu] * w[ju]
    s, d = iu[keep].astype(np.int32), ju[keep].astype(np.int32)
    G = device_graph(n, s, d)
    lagr().lagr_property_tc_lower(G, ctx())
    lrp, lci = lower_csr(G)
    want_rp, want_ci = expected_lower(n, s, d)
    lens = np.diff(want_rp)
    for lo, hi in ((1, 64), (65, 128), (129, 256), (257, 512), (513, 1024), (1025, 2048)):
        assert ((lens >= lo) & (lens <= hi)).any(), (lo, hi)
    assert np.array_equal(lrp, want_rp)
    assert np.array_equal(lci, want_ci)
    A = np.zeros((n, n))
    A[s, d] = A[d, s] = 1.0
    assert lagr().lagr_tc(G, ctx()) == int(round(np.sum((A @ A) * A) / 6))


@pytest.mark.parametrize("entry", GOLD["graphs"], ids=lambda e: f"s{e['scale']}ef{e['edge_factor']}")
def test_tc_rmat_golden(entry):
    n, s, d = rmat(entry["scale"], entry["edge_factor"], entry["seed"])
    G = device_graph(n, s, d)
    assert lagr().lagr_tc(G, ctx()) == entry["triangles"]


def test_tc_small_config_against_oracle_directly():
    n, s, d = rmat(10, 16, 1)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    assert lagr().lagr_tc(G, ctx()) == oracle.triangle_count(rp, ci)


def test_tc_advanced_mode_requires_property():
    L = lagr()
    G, _ = graph_from_edges(*Gs.complete(6))
    with pytest.raises(L.LagrError) as e:
        L.lagr_tc_adv(G, ctx())
    assert e.value.code == L.PROPERTY_MISSING
    L.lagr_property_tc_lower(G, ctx())
    assert L.lagr_tc_adv(G, ctx()) == 20


@pytest.mark.skipif("large" not in GOLD, reason="large golden not generated")
def test_tc_large_config():
    e = GOLD["large"]
    n, s, d = rmat(e["scale"], e["edge_factor"], e["seed"])
    G = device_graph(n, s, d)
    assert lagr().lagr_tc(G, ctx()) == e["triangles"]


@pytest.mark.parametrize("scale,ef,seed", [(10, 16, 1), (14, 16, 103)])
def test_tc_methods_agree_with_the_oracle(scale, ef, seed):
    """lagr_tc's three methods -- the count plan, the fused masked dot of
    lagr_mxm_reduce, and Algorithm 6 as written (C formed by lagr_mxm, then
    reduced) -- all equal the oracle's count; K_12 gives C(12, 3); an
    unknown method is rejected."""
    L = lagr()
    c = ctx()
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    want = oracle.triangle_count(*oracle.build_adjacency(n, s, d))
    for method in (L.TC_DEFAULT, L.TC_DOT, L.TC_MXM, L.TC_DOT, L.TC_DEFAULT):
        assert L.lagr_tc(G, c, method) == want, method
    G, _ = graph_from_edges(*Gs.complete(12))
    assert [L.lagr_tc(G, c, m) for m in (0, 1, 2)] == [220] * 3
    G, _ = graph_from_edges(*Gs.path(9))
    assert [L.lagr_tc(G, c, m) for m in (0, 1, 2)] == [0] * 3
    with pytest.raises(L.LagrError) as e:
        L.lagr_tc(G, c, 3)
    assert e.value.code == L.INVALID_VALUE


@pytest.mark.parametrize("scale,ef,seed", [(18, 8, 41), (18, 16, 42)])
def test_tc_with_hub_columns_matches_the_oracle(scale, ef, seed):
    """Graphs of 2^18 vertices: the count plan keeps pairs with one of the
    1,024 hub columns in row i (ids or bitmap of L_j) or transposes them,
    by cost; the count is checked against the oracle's, and again through
    a batch of this graph and a small one (the packed plan re-bases the
    bitmap entries)."""
    L = lagr()
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    want = oracle.triangle_count(*oracle.build_adjacency(n, s, d))
    assert L.lagr_tc(G, ctx()) == want
    n2, s2, d2 = rmat(9, 8, seed)
    G2 = device_graph(n2, s2, d2)
    B = L.Batch(ctx(), [G2, G])
    got = B.tc(ctx(), L.Tune(8, 4, 0))
    assert got[1] == want and got[0] == oracle.triangle_count(*oracle.build_adjacency(n2, s2, d2))


@pytest.mark.parametrize("n,scale,extra", [((1 << 21) + 4321, 15, 3000000), (5 * (1 << 20) + 77, 15, 4000000),
                                           (13 * (1 << 20) + 5, 14, 4000000)])
def test_tc_cold_columns_over_wide_id_ranges(n, scale, extra):
    """Sparse graphs of 2 to 13 million vertices (R-MAT draws spread over
    the ids plus uniform draws, so most vertices are isolated and the rest
    have labels far apart): the count plan's regions, cursors and item
    table span millions of virtual rows, most of them empty; the counts
    equal the oracle's, and the DOT method's."""
    L = lagr()
    n, s, d = graphgen.spread_edges(n, scale, 16, extra, 7)
    G = device_graph(n, s, d)
    want = oracle.triangle_count(*oracle.build_adjacency(n, s, d))
    assert want > 0
    assert L.lagr_tc(G, ctx()) == want
    assert L.lagr_tc(G, ctx(), L.TC_DOT) == want


@pytest.mark.parametrize("scale,ef,seed", [(12, 4, 11), (13, 8, 12)])
def test_tc_planted_cliques_of_many_widths(scale, ef, seed):
    """Cliques of 5 to 700 vertices planted at random ids of a sparse R-MAT
    graph: after the degree relabel their rows of L are dense prefixes of
    many lengths, so the count plan holds bitmap pairs of many word widths
    (one-width items and items of several widths, whose elements straddle
    pairs at every offset) beside streamed segments in the same items.  The
    count equals the oracle's, the DOT method's and the many-graph batch's."""
    L = lagr()
    n, s, d = rmat(scale, ef, seed)
    rng = np.random.default_rng(seed)
    ss, dd = [np.asarray(s, dtype=np.int64)], [np.asarray(d, dtype=np.int64)]
    for c in (5, 33, 63, 64, 65, 97, 130, 257, 700):
        v = rng.choice(n, size=c, replace=False)
        iu, ju = np.triu_indices(c, 1)
        ss.append(v[iu])
        dd.append(v[ju])
    s2, d2 = np.concatenate(ss), np.concatenate(dd)
    G = device_graph(n, s2, d2)
    want = oracle.triangle_count(*oracle.build_adjacency(n, s2, d2))
    assert want > math.comb(700, 3)
    assert L.lagr_tc(G, ctx()) == want
    assert L.lagr_tc(G, ctx(), L.TC_DOT) == want
    n3, s3, d3 = rmat(8, 8, seed)
    B = L.Batch(ctx(), [device_graph(n3, s3, d3), G])
    got = B.tc(ctx(), L.Tune(8, 4, 0))
    assert got[1] == want and got[0] == oracle.triangle_count(*oracle.build_adjacency(n3, s3, d3))


# ----------------------------------------------------------------- BFS

def bfs_host(G, s, flags=0):
    L = lagr()
    c = ctx()
    lv, pv = L.lagr_bfs(G, s, c, flags)
    return lv.values_full(c).cpu().numpy(), pv.values_full(c).cpu().numpy()


def test_bfs_closed_forms():
    G, (rp, ci) = graph_from_edges(*Gs.path(50))
    lv, pa = bfs_host(G, 0)
    assert lv.tolist() == list(range(50)) and pa.tolist() == [0] + list(range(49))
    r, c = 9, 13
    G, (rp, ci) = graph_from_edges(*Gs.grid(r, c))
    lv, pa = bfs_host(G, 0)
    assert lv.tolist() == [i + j for i in range(r) for j in range(c)]
    check_parents(rp, ci, 0, lv, pa)
    G, _ = graph_from_edges(*Gs.disjoint_union(Gs.cycle(6), Gs.path(4)))
    lv, pa = bfs_host(G, 7)
    assert lv.tolist() == [-1] * 6 + [1, 0, 1, 2]
    assert pa.tolist() == [-1] * 6 + [7, 7, 7, 8]


@pytest.mark.parametrize("scale,ef,seed", [(10, 16, 1), (12, 8, 102), (14, 16, 103)])
def test_bfs_rmat_levels_and_min_parents(scale, ef, seed):
    L = lagr()
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    for src in graphgen.sources(n, s, d, 6, seed):
        src = int(src)
        lv_o, pa_o = oracle.bfs(rp, ci, src)
        mp = oracle.bfs_min_parent(rp, ci, src, lv_o)
        for flags in (0, L.BFS_PUSH_ONLY):
            lv, pa = bfs_host(G, src, flags)
            assert np.array_equal(lv, lv_o.astype(np.int64))
            assert np.array_equal(pa, mp)
        lv, pa = bfs_host(G, src, L.BFS_ANY_PARENT)
        assert np.array_equal(lv, lv_o.astype(np.int64))
        check_parents(rp, ci, src, lv, pa)


def test_bfs_isolated_source_and_bad_source():
    L = lagr()
    G, _ = graph_from_edges(5, [(0, 1), (1, 2)])
    lv, pa = bfs_host(G, 4)
    assert lv.tolist() == [-1, -1, -1, -1, 0] and pa.tolist() == [-1, -1, -1, -1, 4]
    with pytest.raises(L.LagrError) as e:
        L.lagr_bfs(G, 5, ctx())
    assert e.value.code == L.INVALID_INDEX


def test_bfs_large_config_sampled_sources():
    n, s, d = rmat(20, 16, 2)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = graphgen.sources(n, s, d, 64, 2)
    for src in srcs[:3]:
        src = int(src)
        lv_o, _ = oracle.bfs(rp, ci, src)
        mp = oracle.bfs_min_parent(rp, ci, src, lv_o)
        lv, pa = bfs_host(G, src)
        assert np.array_equal(lv, lv_o.astype(np.int64))
        assert np.array_equal(pa, mp)


# ------------------------------------------------------------------ BC

def bc_host(G, sources):
    L = lagr()
    c = ctx()
    return L.lagr_bc(G, sources, c).values_full(c).cpu().numpy()


def test_bc_closed_forms():
    n = 40
    G, _ = graph_from_edges(*Gs.path(n))
    assert_bc_close(bc_host(G, list(range(n))), [2.0 * i * (n - 1 - i) for i in range(n)])
    assert_bc_close(bc_host(G, [0]), [0.0] + [float(n - 1 - i) for i in range(1, n)])
    G, _ = graph_from_edges(*Gs.star(30))
    got = bc_host(G, list(range(30)))
    assert got[0] == 29 * 28 and (got[1:] == 0).all()
    G, _ = graph_from_edges(*Gs.complete(12))
    assert (bc_host(G, list(range(12))) == 0).all()


@pytest.mark.parametrize("scale,ef,seed,ns", [(10, 16, 1, 8), (10, 16, 1, 100), (12, 8, 102, 64),
                                              (14, 16, 103, 64)])
def test_bc_rmat_against_brandes(scale, ef, seed, ns):
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = graphgen.sources(n, s, d, ns, seed)
    assert_bc_close(bc_host(G, srcs), oracle.brandes(rp, ci, srcs))


@pytest.mark.parametrize("scale,ef,seed,ns", [(10, 16, 1, 100), (12, 8, 102, 64), (14, 16, 103, 64)])
def test_bc_backward_push_against_brandes(scale, ef, seed, ns):
    """The backward sweep's push form (W = W B with FP64 atomics), on every
    level and chosen per level, against Brandes at 1e-12 with exact zeros;
    an unknown flag is rejected."""
    L = lagr()
    c = ctx()
    n, s, d = rmat(scale, ef, seed)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = graphgen.sources(n, s, d, ns, seed)
    want = oracle.brandes(rp, ci, srcs)
    for flags in (L.BC_BACKWARD_PUSH_ONLY, L.BC_BACKWARD_PUSH_PULL):
        assert_bc_close(L.lagr_bc(G, srcs, c, flags).values_full(c).cpu().numpy(), want)
    with pytest.raises(L.LagrError) as e:
        L.lagr_bc(G, srcs, c, 4)
    assert e.value.code == L.INVALID_VALUE
    # closed forms through the push: a path and a star
    G, (rp, ci) = graph_from_edges(*Gs.path(30))
    got = L.lagr_bc(G, list(range(30)), c, L.BC_BACKWARD_PUSH_ONLY).values_full(c).cpu().numpy()
    assert_bc_close(got, oracle.brandes(rp, ci, np.arange(30)))
    G, (rp, ci) = graph_from_edges(*Gs.star(3000))
    got = L.lagr_bc(G, list(range(64)), c, L.BC_BACKWARD_PUSH_ONLY).values_full(c).cpu().numpy()
    assert_bc_close(got, oracle.brandes(rp, ci, np.arange(64)))


def test_bc_duplicate_and_isolated_sources():
    G, (rp, ci) = graph_from_edges(8, [(0, 1), (1, 2), (2, 3), (3, 0), (2, 4)])
    srcs = [2, 2, 7, 0]
    assert_bc_close(bc_host(G, srcs), oracle.brandes(rp, ci, srcs))


def test_bc_large_config_one_batch():
    n, s, d = rmat(18, 16, 3)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = graphgen.sources(n, s, d, 256, 3)[:64]
    assert_bc_close(bc_host(G, srcs), oracle.brandes(rp, ci, srcs))


def test_bfs_batch_ragged_duplicate_and_isolated_sources():
    """lagr_bfs_batch over 70 sources (a full block of 64 and a ragged one),
    with a repeated source and an isolated one, against the queue BFS; a
    directed graph and a bad source are rejected."""
    L = lagr()
    c = ctx()
    n, s, d = rmat(12, 8, 102)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    deg = np.diff(rp)
    iso = int(np.nonzero(deg == 0)[0][0])
    srcs = [int(x) for x in graphgen.sources(n, s, d, 68, 7)] + [iso]
    srcs.insert(5, srcs[3])
    lev, reached, lsum, depth = L.lagr_bfs_batch(G, srcs, c)
    assert lev.shape == (70, n)
    for k, src in enumerate(srcs):
        ref, _ = oracle.bfs(rp, ci, src)
        assert np.array_equal(lev[k].cpu().numpy(), ref), src
        r = ref >= 0
        assert (reached[k], lsum[k], depth[k]) == (int(r.sum()), int(ref[r].sum()), int(ref.max()))
    _, reached_only, _, _ = L.lagr_bfs_batch(G, srcs[:3], c, want_levels=False)
    assert list(reached_only) == list(reached[:3])
    with pytest.raises(L.LagrError) as e:
        L.lagr_bfs_batch(G, [n], c)
    assert e.value.code == L.INVALID_INDEX
    A = L.Matrix.build(c, 4, 4, torch.tensor([0, 1], dtype=torch.int32).cuda(),
                       torch.tensor([1, 2], dtype=torch.int32).cuda(), 0)
    D = L.Graph(c, A, L.ADJACENCY_DIRECTED)
    with pytest.raises(L.LagrError) as e:
        L.lagr_bfs_batch(D, [0], c)
    assert e.value.code == L.INVALID_VALUE


def test_tc_and_bfs_autotune_keep_results():
    """The tuners time their candidates on the device and keep the fastest
    in the graph: the hub count is one of the candidates, the thresholds
    one of the grid's pairs, and counts, levels and parents after tuning
    (and after dropping the cached properties) equal the oracle's."""
    L = lagr()
    c = ctx()
    n, s, d = rmat(14, 16, 103)
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    want = oracle.triangle_count(rp, ci)
    hubs = L.lagr_tc_autotune(G, c)
    assert hubs in {0} | {min(n >> k, 4096) for k in range(7, 11)}
    assert L.lagr_tc(G, c) == want
    G.delete_properties(c)
    assert L.lagr_tc(G, c) == want
    srcs = [int(x) for x in graphgen.sources(n, s, d, 4, 103)]
    a, b = L.lagr_bfs_autotune(G, srcs, c)
    assert a in (6, 10, 14, 20, 32) and b in (12, 24, 48)
    for src in srcs:
        lv_o, _ = oracle.bfs(rp, ci, src)
        lv, pa = bfs_host(G, src)
        assert np.array_equal(lv, lv_o.astype(np.int64))
        assert np.array_equal(pa, oracle.bfs_min_parent(rp, ci, src, lv_o))
    with pytest.raises(L.LagrError) as e:
        L.lagr_bfs_autotune(G, [], c)
    assert e.value.code == L.INVALID_VALUE
    assert G.tuning() == (hubs, a, b)
    # set by hand: a new hub count (other than the tuner's choice) drops the
    # operand, which is rebuilt
    other = 0 if hubs != 0 else min(n >> 8, 4096)
    G.set_tuning(c, other, 32, -1)
    assert G.tuning() == (other, 32, b) and G.tc_lower() is None
    assert L.lagr_tc(G, c) == want
    lv, _ = bfs_host(G, srcs[0])
    assert np.array_equal(lv, oracle.bfs(rp, ci, srcs[0])[0].astype(np.int64))
    for bad in ((-2, -1, -1), (-1, 0, -1), (-1, -1, -5)):
        with pytest.raises(L.LagrError) as e:
            G.set_tuning(c, *bad)
        assert e.value.code == L.INVALID_VALUE
