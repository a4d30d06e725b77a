"""ORACLE -- test infrastructure, not part of the product.

A plain CPU statement of what the device library computes, written from the
paper (LAGraph, arXiv 2104.01661): triangle counting (Section IV-E,
Algorithm 6), breadth-first search (Section IV-A, Algorithms 1-2), Brandes
betweenness centrality (Section IV-B, Algorithm 3), and the shortest-path
distances of delta-stepping (Section IV-D, Algorithm 5) by Dijkstra's
algorithm, directed graphs (the transpose property AT, BFS parents and
Brandes over in-edges), PageRank (Section IV-C, Algorithm 4) and connected
components (Section IV-F, Algorithm 7) in ``oracle.c``, and the
GraphBLAS masked-product / accumulate / reduce semantics of Section III
(Table I, Table II, "Masks") as a dense brute-force reference in
``semantics.py``.

Only ``tests/``, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the device path; the only
common dependency is the seeded input generator ``graphgen``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SO_MT = os.path.join(_HERE, "liboracle_mt.so")
_SRC = os.path.join(_HERE, "oracle.c")


def build(force: bool = False) -> str:
    """Compile the C oracle: the checker (plain -O2, single-threaded) and,
    from the same source, the timing build of the CPU baseline (-O3
    -march=native, OpenMP over independent units in the timing drivers)."""
    for so, flags in ((_SO, ["-O2"]), (_SO_MT, ["-O3", "-march=native", "-fopenmp"])):
        if force or not os.path.exists(so) or os.path.getmtime(so) < os.path.getmtime(_SRC):
            tmp = so + ".tmp"
            subprocess.check_call(["gcc", *flags, "-fPIC", "-shared", _SRC, "-o", tmp])
            os.replace(tmp, so)
    return _SO


_lib = None
_P = ctypes.c_void_p
_I = ctypes.c_int64


def _declare(lib):
    lib.orc_threads.restype = ctypes.c_int
    lib.orc_threads.argtypes = []
    lib.orc_set_threads.restype = None
    lib.orc_set_threads.argtypes = [ctypes.c_int]
    lib.orc_tc_par.restype = _I
    lib.orc_tc_par.argtypes = [_I, _P, _P, _I]
    lib.orc_bfs_sources.restype = ctypes.c_int
    lib.orc_bfs_sources.argtypes = [_I, _P, _P, _I, _P, _P, _P]
    lib.orc_brandes_parts.restype = ctypes.c_int
    lib.orc_brandes_parts.argtypes = [_I, _P, _P, _I, _P, _I, _P, _P]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        _declare(lib)
        lib.orc_build.restype = _I
        lib.orc_build.argtypes = [_I, _I, _P, _P, _P, _P]
        lib.orc_tc.restype = _I
        lib.orc_tc.argtypes = [_I, _P, _P]
        lib.orc_tc_rows.restype = _I
        lib.orc_tc_rows.argtypes = [_I, _P, _P, _I, _I, _I]
        lib.orc_tc_lower_counts.restype = _I
        lib.orc_tc_lower_counts.argtypes = [_I, _P, _P, _P, _P, _P]
        lib.orc_bfs.restype = ctypes.c_int
        lib.orc_bfs.argtypes = [_I, _P, _P, _I, _P, _P]
        lib.orc_bfs_min_parent.restype = None
        lib.orc_bfs_min_parent.argtypes = [_I, _P, _P, _I, _P, _P]
        lib.orc_brandes.restype = ctypes.c_int
        lib.orc_brandes.argtypes = [_I, _P, _P, _I, _P, _P]
        lib.orc_dijkstra.restype = ctypes.c_int
        lib.orc_dijkstra.argtypes = [_I, _P, _P, _P, _I, _P]
        lib.orc_build_directed.restype = _I
        lib.orc_build_directed.argtypes = [_I, _I, _P, _P, _P, _P]
        lib.orc_transpose.restype = ctypes.c_int
        lib.orc_transpose.argtypes = [_I, _I, _P, _P, _P, _P, _P]
        lib.orc_brandes_directed.restype = ctypes.c_int
        lib.orc_brandes_directed.argtypes = [_I, _P, _P, _P, _P, _I, _P, _P]
        lib.orc_pagerank.restype = _I
        lib.orc_pagerank.argtypes = [_I, _P, _P, _P, ctypes.c_double, ctypes.c_double, _I, _P]
        lib.orc_components.restype = ctypes.c_int
        lib.orc_components.argtypes = [_I, _P, _P, _P, _P, _P]
        _lib = lib
    return _lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a, a.ctypes.data


def build_adjacency(n: int, src, dst):
    """Undirected adjacency from raw edge draws: both directions, no
    self-loops, rows sorted, duplicates removed.  -> (rowptr int64[n+1],
    colidx int32[nnz])."""
    src, ps = _c(src, np.int32)
    dst, pd = _c(dst, np.int32)
    rowptr = np.empty(n + 1, dtype=np.int64)
    colidx = np.empty(max(2 * src.size, 1), dtype=np.int32)
    nnz = _load().orc_build(n, src.size, ps, pd, rowptr.ctypes.data, colidx.ctypes.data)
    if nnz < 0:
        raise MemoryError("oracle: graph build failed")
    return rowptr, colidx[:nnz].copy()


def from_edges(n: int, pairs):
    """Adjacency of a small graph given as an iterable of (u, v) pairs."""
    pairs = list(pairs)
    src = np.array([p[0] for p in pairs], dtype=np.int32)
    dst = np.array([p[1] for p in pairs], dtype=np.int32)
    return build_adjacency(n, src, dst)


def triangle_count(rowptr, colidx) -> int:
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    return int(_load().orc_tc(rowptr.size - 1, pr, pc))


def triangle_count_rows(rowptr, colidx, u0: int, u1: int, stride: int = 1) -> int:
    """Triangles whose smallest vertex is one of u0, u0+stride, ... < u1."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    return int(_load().orc_tc_rows(rowptr.size - 1, pr, pc, u0, u1, stride))


def lower_counts(rowptr, colidx):
    """C<s(L)> = L plus.pair L' entry by entry -> (Lrowptr, Lcolidx, C values)."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    n = rowptr.size - 1
    cap = max(colidx.size // 2 + 1, 1)
    lrp = np.empty(n + 1, dtype=np.int64)
    lci = np.empty(cap, dtype=np.int32)
    cnt = np.empty(cap, dtype=np.int64)
    q = _load().orc_tc_lower_counts(n, pr, pc, lrp.ctypes.data, lci.ctypes.data, cnt.ctypes.data)
    return lrp, lci[:q].copy(), cnt[:q].copy()


def bfs(rowptr, colidx, source: int):
    """FIFO-queue BFS -> (level int32[n], parent int64[n]); -1 = unreached."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    n = rowptr.size - 1
    level = np.empty(n, dtype=np.int32)
    parent = np.empty(n, dtype=np.int64)
    if _load().orc_bfs(n, pr, pc, int(source), level.ctypes.data, parent.ctypes.data) != 0:
        raise MemoryError("oracle: bfs failed")
    return level, parent


def bfs_min_parent(rowptr, colidx, source: int, level):
    """Deterministic parents: smallest neighbour one level closer."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    level, pl = _c(level, np.int32)
    parent = np.empty(rowptr.size - 1, dtype=np.int64)
    _load().orc_bfs_min_parent(rowptr.size - 1, pr, pc, int(source), pl, parent.ctypes.data)
    return parent


def brandes(rowptr, colidx, sources):
    """Unnormalised betweenness summed over `sources` (FP64)."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    srcs, ps = _c(sources, np.int64)
    out = np.empty(rowptr.size - 1, dtype=np.float64)
    rc = _load().orc_brandes(rowptr.size - 1, pr, pc, srcs.size, ps, out.ctypes.data)
    if rc == -2:
        raise OverflowError("oracle: a shortest-path count reached 2^53")
    if rc != 0:
        raise MemoryError("oracle: brandes failed")
    return out


def build_directed(n: int, src, dst):
    """Directed adjacency from raw edge draws: (src[e], dst[e]) is the edge
    src -> dst; no self-loops, rows sorted, duplicates removed."""
    src, ps = _c(src, np.int32)
    dst, pd = _c(dst, np.int32)
    rowptr = np.empty(n + 1, dtype=np.int64)
    colidx = np.empty(max(src.size, 1), dtype=np.int32)
    nnz = _load().orc_build_directed(n, src.size, ps, pd, rowptr.ctypes.data, colidx.ctypes.data)
    if nnz < 0:
        raise MemoryError("oracle: graph build failed")
    return rowptr, colidx[:nnz].copy()


def transpose(rowptr, colidx, ncols=None, values=None):
    """Transpose of a CSR (rows sorted) -> (rowptr, colidx) or, with values,
    (rowptr, colidx, values)."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    nrows = rowptr.size - 1
    ncols = nrows if ncols is None else int(ncols)
    rpT = np.empty(ncols + 1, dtype=np.int64)
    ciT = np.empty(max(colidx.size, 1), dtype=np.int32)
    perm = np.empty(max(colidx.size, 1), dtype=np.int64)
    if _load().orc_transpose(nrows, ncols, pr, pc, rpT.ctypes.data, ciT.ctypes.data, perm.ctypes.data) != 0:
        raise MemoryError("oracle: transpose failed")
    ciT, perm = ciT[:colidx.size].copy(), perm[:colidx.size]
    if values is None:
        return rpT, ciT
    return rpT, ciT, np.asarray(values)[perm]


def brandes_directed(rowptr, colidx, sources):
    """Unnormalised betweenness of a directed graph summed over `sources`:
    paths follow out-edges, the backward sweep reads in-edges (FP64)."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    rpT, ciT = transpose(rowptr, colidx)
    rpT, prT = _c(rpT, np.int64)
    ciT, pcT = _c(ciT, np.int32)
    srcs, ps = _c(sources, np.int64)
    out = np.empty(rowptr.size - 1, dtype=np.float64)
    rc = _load().orc_brandes_directed(rowptr.size - 1, pr, pc, prT, pcT, srcs.size, ps, out.ctypes.data)
    if rc == -2:
        raise OverflowError("oracle: a shortest-path count reached 2^53")
    if rc != 0:
        raise MemoryError("oracle: brandes failed")
    return out


def pagerank(rowptr, colidx, damping=0.85, tol=1e-4, itermax=100):
    """PageRank as Algorithm 4 (GAP) states it -> (rank float64[n],
    iterations).  Rows of (rowptr, colidx) are out-edges."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    n = rowptr.size - 1
    rpT, ciT = transpose(rowptr, colidx)
    rpT, prT = _c(rpT, np.int64)
    ciT, pcT = _c(ciT, np.int32)
    dout, pd = _c(np.diff(rowptr), np.int64)
    r = np.empty(n, dtype=np.float64)
    k = _load().orc_pagerank(n, prT, pcT, pd, float(damping), float(tol), int(itermax), r.ctypes.data)
    if k < 0:
        raise MemoryError("oracle: pagerank failed")
    return r, int(k)


def components(rowptr, colidx, directed=False):
    """Label of every vertex = the smallest vertex id of its (weakly)
    connected component (int64[n])."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    if directed:
        rpT, ciT = transpose(rowptr, colidx)
        rpT, prT = _c(rpT, np.int64)
        ciT, pcT = _c(ciT, np.int32)
    else:
        prT, pcT = pr, pc
    label = np.empty(rowptr.size - 1, dtype=np.int64)
    if _load().orc_components(rowptr.size - 1, pr, pc, prT, pcT, label.ctypes.data) != 0:
        raise MemoryError("oracle: components failed")
    return label


def dijkstra(rowptr, colidx, weights, source: int):
    """Shortest-path distances from source (float64[n], +inf unreached);
    weights: one non-negative float64 per CSR entry."""
    rowptr, pr = _c(rowptr, np.int64)
    colidx, pc = _c(colidx, np.int32)
    weights, pw = _c(weights, np.float64)
    out = np.empty(rowptr.size - 1, dtype=np.float64)
    if _load().orc_dijkstra(rowptr.size - 1, pr, pc, pw, int(source), out.ctypes.data) != 0:
        raise MemoryError("oracle: dijkstra failed")
    return out


# ------------------------------------------------------------ timing build

class Timing:
    """The timing build of the oracle (the same C source, -O3 -march=native,
    OpenMP over independent units) or, with threaded=False, the checker
    library itself.  Used by the benchmark's CPU-baseline leg only."""

    def __init__(self, threaded: bool = True):
        if threaded:
            if not os.path.exists(_SO_MT) or os.path.getmtime(_SO_MT) < os.path.getmtime(_SRC):
                build()
            self.lib = ctypes.CDLL(_SO_MT)
            _declare(self.lib)
        else:
            self.lib = _load()

    def threads(self) -> int:
        return int(self.lib.orc_threads())

    def set_threads(self, t: int):
        self.lib.orc_set_threads(int(t))

    def triangle_count(self, rowptr, colidx, stride: int = 1) -> int:
        """Triangles whose smallest vertex is one of 0, stride, 2 stride, ..."""
        rowptr, pr = _c(rowptr, np.int64)
        colidx, pc = _c(colidx, np.int32)
        return int(self.lib.orc_tc_par(rowptr.size - 1, pr, pc, int(stride)))

    def bfs_sources(self, rowptr, colidx, sources):
        """(levels int32[ns, n], smallest parents int64[ns, n])."""
        rowptr, pr = _c(rowptr, np.int64)
        colidx, pc = _c(colidx, np.int32)
        srcs, ps = _c(sources, np.int64)
        n = rowptr.size - 1
        lv = np.empty((srcs.size, n), dtype=np.int32)
        pa = np.empty((srcs.size, n), dtype=np.int64)
        if self.lib.orc_bfs_sources(n, pr, pc, srcs.size, ps, lv.ctypes.data, pa.ctypes.data) != 0:
            raise MemoryError("oracle: bfs failed")
        return lv, pa

    def brandes(self, rowptr, colidx, sources, nparts: int):
        rowptr, pr = _c(rowptr, np.int64)
        colidx, pc = _c(colidx, np.int32)
        srcs, ps = _c(sources, np.int64)
        n = rowptr.size - 1
        part = np.empty((max(1, nparts), n), dtype=np.float64)
        out = np.empty(n, dtype=np.float64)
        rc = self.lib.orc_brandes_parts(n, pr, pc, srcs.size, ps, int(nparts), part.ctypes.data,
                                        out.ctypes.data)
        if rc == -2:
            raise OverflowError("oracle: a shortest-path count reached 2^53")
        if rc != 0:
            raise MemoryError("oracle: brandes failed")
        return out
