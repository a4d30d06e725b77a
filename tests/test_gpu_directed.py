"""Directed graphs through the C ABI: the cached transpose (the AT property),
direction-optimising BFS whose pull steps read AT, batched BC whose pull
steps read AT and whose backward sweep reads A, and Algorithm 2's identity
of push and pull (vxm with A, and with AT under the transpose descriptor)
on a graph that is not symmetric.  Checked against the oracle's directed
build, transpose, queue BFS, in-neighbour parents and directed Brandes."""
import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_util import assert_bc_close, ctx, lagr

pytestmark = pytest.mark.gpu


def device_digraph(n, s, d):
    L = lagr()
    c = ctx()
    A = L.Matrix.build(c, n, n, torch.from_numpy(np.ascontiguousarray(s, np.int32)).cuda(),
                       torch.from_numpy(np.ascontiguousarray(d, np.int32)).cuda(), L.BUILD_DROP_LOOPS)
    G = L.Graph(c, A, L.ADJACENCY_DIRECTED)
    G.check(c)
    return G


def csr_of(M):
    rp, ci, vals = M.to_csr(ctx())
    return rp.cpu().numpy(), ci.cpu().numpy(), None if vals is None else vals.cpu().numpy()


@pytest.mark.parametrize("scale,ef,seed", [(8, 8, 201), (11, 16, 202)])
def test_device_build_and_transpose_equal_the_oracle(scale, ef, seed):
    L = lagr()
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    G = device_digraph(n, s, d)
    rp, ci, _ = csr_of(G.matrix())
    orp, oci = oracle.build_directed(n, s, d)
    assert np.array_equal(rp, orp) and np.array_equal(ci, oci)
    with pytest.raises(L.LagrError) as e:
        G.at()
    assert e.value.code == L.PROPERTY_MISSING
    G.property_at(ctx())
    trp, tci, _ = csr_of(G.at())
    wrp, wci = oracle.transpose(orp, oci)
    assert np.array_equal(trp, wrp) and np.array_equal(tci, wci)
    G.delete_properties(ctx())
    with pytest.raises(L.LagrError):
        G.at()


def test_weighted_transpose_carries_values_and_undirected_is_its_own():
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(9, 8, 203)
    rp, ci = oracle.build_directed(n, s, d)
    w = np.arange(1, ci.size + 1, dtype=np.float64) * 0.5
    A = L.Matrix.wrap_csr(c, n, n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                          torch.from_numpy(w).cuda())
    G = L.Graph(c, A, L.ADJACENCY_DIRECTED)
    G.property_at(c)
    trp, tci, tw = csr_of(G.at())
    wrp, wci, ww = oracle.transpose(rp, ci, values=w)
    assert np.array_equal(trp, wrp) and np.array_equal(tci, wci) and np.array_equal(tw, ww)
    urp, uci = oracle.build_adjacency(n, s, d)
    U = L.Graph(c, L.Matrix.wrap_csr(c, n, n, torch.from_numpy(urp).cuda(), torch.from_numpy(uci).cuda()))
    U.property_at(c)                                   # no-op: A is its own transpose
    arp, aci, _ = csr_of(U.at())
    assert np.array_equal(arp, urp) and np.array_equal(aci, uci)


@pytest.mark.parametrize("scale,ef,seed", [(10, 8, 204), (14, 16, 205)])
def test_directed_bfs_levels_and_smallest_in_neighbour_parents(scale, ef, seed):
    L = lagr()
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    G = device_digraph(n, s, d)
    rp, ci = oracle.build_directed(n, s, d)
    rpT, ciT = oracle.transpose(rp, ci)
    for flags in (0, L.BFS_PUSH_ONLY):
        for src in graphgen.sources(n, s, d, 4, seed):
            src = int(src)
            lv, pv = L.lagr_bfs(G, src, ctx(), flags)
            level = lv.values_full(ctx()).cpu().numpy()
            parent = pv.values_full(ctx()).cpu().numpy()
            olev, _ = oracle.bfs(rp, ci, src)
            assert np.array_equal(level, olev.astype(np.int64)), (src, flags)
            assert np.array_equal(parent, oracle.bfs_min_parent(rpT, ciT, src, olev)), (src, flags)


def test_directed_bfs_any_parent_is_a_valid_in_neighbour():
    L = lagr()
    n, s, d = graphgen.rmat_edges(13, 16, 206)
    G = device_digraph(n, s, d)
    rp, ci = oracle.build_directed(n, s, d)
    for src in graphgen.sources(n, s, d, 3, 7):
        src = int(src)
        lv, pv = L.lagr_bfs(G, src, ctx(), L.BFS_ANY_PARENT)
        level = lv.values_full(ctx()).cpu().numpy()
        parent = pv.values_full(ctx()).cpu().numpy()
        olev, _ = oracle.bfs(rp, ci, src)
        assert np.array_equal(level, olev.astype(np.int64))
        assert parent[src] == src and (parent[level < 0] == -1).all()
        v = np.nonzero(level > 0)[0]
        p = parent[v]
        assert (level[p] == level[v] - 1).all()
        for pp, vv in zip(p, v):                       # edge p -> v exists
            row = ci[rp[pp]:rp[pp + 1]]
            k = np.searchsorted(row, vv)
            assert k < row.size and row[k] == vv


@pytest.mark.parametrize("scale,ef,seed,ns", [(9, 8, 207, 70), (12, 16, 208, 128)])
def test_directed_bc_matches_directed_brandes(scale, ef, seed, ns):
    L = lagr()
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    G = device_digraph(n, s, d)
    rp, ci = oracle.build_directed(n, s, d)
    srcs = graphgen.sources(n, s, d, ns, seed)
    got = L.lagr_bc(G, srcs, ctx()).values_full(ctx()).cpu().numpy()
    want = oracle.brandes_directed(rp, ci, srcs)
    assert_bc_close(got, want)
    # the backward push scatters over in-edges (rows of AT)
    for flags in (L.BC_BACKWARD_PUSH_ONLY, L.BC_BACKWARD_PUSH_PULL):
        assert_bc_close(L.lagr_bc(G, srcs, ctx(), flags).values_full(ctx()).cpu().numpy(), want)


def test_push_and_pull_levels_agree_on_a_directed_graph():
    """Algorithm 2: q<!s(p)> = q any.secondi A (push) equals the same product
    with AT under the transpose descriptor (pull), level by level."""
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(10, 8, 209)
    G = device_digraph(n, s, d)
    G.property_at(c)
    A, AT = G.matrix(), G.at()
    src = int(graphgen.sources(n, s, d, 1, 3)[0])
    idx = torch.tensor([src], dtype=torch.int32, device="cuda")
    val = torch.tensor([src], dtype=torch.int64, device="cuda")
    frontier = {}
    for name, M, desc in (("push", A, L.DESC_RSC), ("pull", AT, L.DESC_RSC | L.DESC_TRAN1)):
        q = L.Vector.wrap_sparse(c, n, idx.clone(), val.clone(), typ=L.INT64)
        p = L.Vector.wrap_sparse(c, n, idx.clone(), val.clone(), typ=L.INT64)
        levels = []
        for _ in range(n):
            L.lagr_vxm(q, p, 0, L.ANY_SECONDI, q, M, desc | L.DESC_ASSIGN_PARENT, c)
            qi, _ = q.to_tuples(c)
            if qi.numel() == 0:
                break
            levels.append(sorted(qi.cpu().numpy().tolist()))
        frontier[name] = levels
    assert frontier["push"] == frontier["pull"] and len(frontier["push"]) > 2
    rp, ci = oracle.build_directed(n, s, d)
    olev, _ = oracle.bfs(rp, ci, src)
    for k, lev in enumerate(frontier["push"], start=1):
        assert lev == np.nonzero(olev == k)[0].tolist()
