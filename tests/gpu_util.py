"""Helpers for the GPU tests: device graphs from seeded inputs, checks."""
from __future__ import annotations

import numpy as np
import torch

import graphgen
import oracle


def lagr():
    from paper_2104_01661_amd import lagr as L
    return L


_CTX = None


def ctx():
    global _CTX
    if _CTX is None:
        L = lagr()
        L.use_torch_allocator(True)
        _CTX = L.Context(0)
    return _CTX


def device_graph(n, src, dst):
    """Undirected graph built on the device from raw draws (both directions,
    no self-loops, duplicates collapsed), checked."""
    L = lagr()
    c = ctx()
    s = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int32)).cuda()
    d = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.int32)).cuda()
    A = L.Matrix.build(c, n, n, s, d, L.BUILD_SYMMETRIZE | L.BUILD_DROP_LOOPS)
    G = L.Graph(c, A)
    G.check(c)
    return G


def graph_from_edges(n, edges):
    e = list(edges)
    src = np.array([u for u, _ in e], dtype=np.int32)
    dst = np.array([v for _, v in e], dtype=np.int32)
    return device_graph(n, src, dst), oracle.from_edges(n, e)


def rmat(scale, ef, seed):
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    return n, s, d


def graph_csr(G):
    """(rowptr, colidx) of a device graph's adjacency, on the host."""
    L = lagr()
    import ctypes
    h = ctypes.c_void_p()
    L.call("lagr_graph_matrix", ctypes.byref(h), G.h)
    M = L.Matrix(h)
    rp, ci, _ = M.to_csr(ctx())
    M.h = ctypes.c_void_p()   # borrowed from the graph: do not free
    return rp.cpu().numpy(), ci.cpu().numpy()


def check_parents(rp, ci, s, level, parent):
    """Vectorised BFS-tree validity: parent(s)=s, unreached -1, and every
    other reached v has an edge to a parent one level closer."""
    n = rp.size - 1
    assert parent[s] == s and level[s] == 0
    un = level < 0
    assert (parent[un] == -1).all()
    v = np.nonzero(~un)[0]
    v = v[v != s]
    p = parent[v]
    assert (p >= 0).all()
    assert (level[p] == level[v] - 1).all()
    # edge (p, v) exists: binary search v in row p
    for pv, vv in zip(p, v):
        row = ci[rp[pv]:rp[pv + 1]]
        k = np.searchsorted(row, vv)
        assert k < row.size and row[k] == vv


def assert_bc_close(got, want, rtol=1e-12):
    got = np.asarray(got)
    want = np.asarray(want)
    zero = want == 0
    assert (got[zero] == 0).all(), "nonzero score where the oracle has exactly 0"
    nz = ~zero
    err = np.abs(got[nz] - want[nz]) / np.abs(want[nz])
    assert err.size == 0 or err.max() <= rtol, f"max rel err {err.max():.3e}"


def bfs_graphblas(c, A, AT, n, src, mode="auto", alpha=14, beta=24):
    """Algorithms 1-2 written with lagr_vxm: q<!s(p), r> = q any.secondi A
    (push), or the same product over AT under TRAN1 (pull), each with the
    parents assigned into p in the same call.  mode "push" is Algorithm 1;
    "auto" switches direction by Beamer's test on the two entry counts.
    Returns the parent array (-1 unreached) and the number of levels."""
    L = lagr()
    idx = torch.tensor([src], dtype=torch.int32, device="cuda")
    val = torch.tensor([src], dtype=torch.int64, device="cuda")
    q = L.Vector.wrap_sparse(c, n, idx, val, typ=L.INT64)
    p = L.Vector.wrap_sparse(c, n, idx.clone(), val.clone(), typ=L.INT64)
    pull, nq, nvisited, levels = False, 1, 1, 0
    while nq > 0:
        if mode == "auto":
            if not pull and nq > (n - nvisited) / alpha:
                pull = True
            elif pull and nq < n / beta:
                pull = False
        if pull:
            L.lagr_vxm(q, p, 0, L.ANY_SECONDI, q, AT, L.DESC_RSC | L.DESC_TRAN1 | L.DESC_ASSIGN_PARENT, c)
        else:
            L.lagr_vxm(q, p, 0, L.ANY_SECONDI, q, A, L.DESC_RSC | L.DESC_ASSIGN_PARENT, c)
        nq = q.nvals(c)
        nvisited += nq
        levels += 1
    pres, vals = p.to_dense(c, fill=-1)
    return vals.cpu().numpy(), levels - 1
