"""Seeded synthetic inputs shared by the oracle and the device path.

Holds none of the method's arithmetic: R-MAT raw edge draws (Chakrabarti,
Zhan and Faloutsos 2004) with the a/b/c/d = .57/.19/.19/.05 split, seeded
source sampling and the workload recipes (sizes, seeds, query streams).  The
adjacency matrix is built from the raw draws separately by each side.

The paper measures on the GAP benchmark graphs (Table IV); those are not
available here, so seeded R-MAT graphs of the same power-law Kronecker
family stand in for them.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_SRC = os.path.join(_HERE, "rmat.c")

RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19

TAG_EDGES = 0
TAG_SOURCES = 0x737263          # "src"
TAG_PARAMS = 0x70726d           # "prm"
TAG_QUERIES = 0x717279          # "qry"
TAG_WEIGHTS = 0x777467          # "wtg"
TAG_SPREAD = 0x737072           # "spr"


def build(force: bool = False) -> str:
    """Compile the generator with gcc (OpenMP over independent draws)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", _SRC, "-o", tmp])
        os.replace(tmp, _SO)
    return _SO


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        lib.gg_splitmix64.restype = ctypes.c_uint64
        lib.gg_splitmix64.argtypes = [ctypes.c_uint64]
        lib.gg_rmat_edges.restype = None
        lib.gg_rmat_edges.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_uint64,
                                      ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_touched.restype = None
        lib.gg_touched.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]
        lib.gg_sample.restype = ctypes.c_int
        lib.gg_sample.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_uint64,
                                  ctypes.c_uint64, ctypes.c_void_p]
        lib.gg_edge_weights.restype = None
        lib.gg_edge_weights.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                        ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        lib.gg_uniforms.restype = None
        lib.gg_uniforms.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                    ctypes.c_int64, ctypes.c_void_p]
        _lib = lib
    return _lib


def splitmix64(x: int) -> int:
    return int(_load().gg_splitmix64(ctypes.c_uint64(x & 0xFFFFFFFFFFFFFFFF)))


def rmat_edges(scale: int, edge_factor: int, seed: int,
               a: float = RMAT_A, b: float = RMAT_B, c: float = RMAT_C):
    """Raw R-MAT draws: (n, src int32[m], dst int32[m]) with m = ef * 2^scale.

    Self-loops and duplicate pairs are kept; nothing is symmetrised."""
    n = 1 << scale
    m = edge_factor * n
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    _load().gg_rmat_edges(scale, m, seed, a, b, c, src.ctypes.data, dst.ctypes.data)
    return n, src, dst


def spread_edges(n: int, scale: int, edge_factor: int, extra: int, seed: int, step: int = 1000003):
    """Raw draws on n >= 2^scale vertices: R-MAT draws of the given scale
    placed by v -> v * step mod n (one-to-one: step is a prime that must not
    divide n), then `extra` uniform draws over all n vertices.  A sparse
    graph whose non-isolated vertices spread over a wide id range."""
    if n < (1 << scale) or n % step == 0:
        raise ValueError("n must be at least 2^scale and not a multiple of step")
    _, s, d = rmat_edges(scale, edge_factor, seed)
    s = (s.astype(np.int64) * step) % n
    d = (d.astype(np.int64) * step) % n
    u = uniforms(seed, TAG_SPREAD, 2 * extra)
    us = np.minimum((u[:extra] * n).astype(np.int64), n - 1)
    ud = np.minimum((u[extra:] * n).astype(np.int64), n - 1)
    return n, np.concatenate([s, us]).astype(np.int32), np.concatenate([d, ud]).astype(np.int32)


def touched_vertices(n: int, src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Vertices that appear in at least one draw with u != v (non-isolated
    once the graph is built), ascending int64."""
    flag = np.empty(n, dtype=np.uint8)
    _load().gg_touched(n, src.size, src.ctypes.data, dst.ctypes.data, flag.ctypes.data)
    return np.nonzero(flag)[0].astype(np.int64)


def sample(candidates: np.ndarray, k: int, seed: int, tag: int = TAG_SOURCES) -> np.ndarray:
    """k distinct elements of `candidates`, drawn without replacement."""
    pos = np.empty(k, dtype=np.int64)
    rc = _load().gg_sample(candidates.size, k, seed, tag, pos.ctypes.data)
    if rc != 0:
        raise ValueError(f"cannot draw {k} of {candidates.size} candidates")
    return candidates[pos]


def uniforms(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().gg_uniforms(seed, tag, start, count, out.ctypes.data)
    return out


def edge_weights(rowptr, colidx, seed: int, wmax: int = 255) -> np.ndarray:
    """Symmetric seeded integer weights in [1, wmax] (as float64), one per
    CSR entry: w(u, v) = w(v, u)."""
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    out = np.empty(ci.size, dtype=np.float64)
    _load().gg_edge_weights(rp.size - 1, rp.ctypes.data, ci.ctypes.data, seed, TAG_WEIGHTS, wmax,
                            out.ctypes.data)
    return out


def sources(n: int, src: np.ndarray, dst: np.ndarray, k: int, seed: int) -> np.ndarray:
    """k seeded distinct non-isolated sources (draw order kept)."""
    return sample(touched_vertices(n, src, dst), k, seed, TAG_SOURCES)


# --------------------------------------------------------------------------
# Workload recipes
# --------------------------------------------------------------------------

TC_SMALL = dict(name="rmat-s10-ef16-tc", scale=10, edge_factor=16, seed=1)
LARGE = dict(name="rmat-s20-ef16-tc+dobfs64", scale=20, edge_factor=16, seed=2, bfs_sources=64)
BC = dict(name="rmat-s18-ef16-bc4x64", scale=18, edge_factor=16, seed=3, batches=4, batch_size=64)
# delta-stepping SSSP on the LARGE graph with symmetric integer weights 1..255
SSSP = dict(name="rmat-s20-ef16-sssp8-w1..255", weight_seed=20, wmax=255, sources=8, source_seed=21,
            deltas=(16.0, 32.0, 64.0, 128.0))
MANY = dict(name="rmat-2000-graphs-s8..16", count=2000, base=4 << 32)
SERVE = dict(name="serve-32-graphs-s12..22", count=32, base=5 << 32, rate=5000.0,
             mix=(0.3, 0.5, 0.2), bc_sources=8, budget_bytes=64 << 30, stream_seed=55)


def many_graph_params(g: int):
    """(scale, edge_factor, seed) of graph g of the many-graph batch:
    scale uniform in 8..16, edge factor uniform in {4, 8, 16, 32}."""
    seed = splitmix64(MANY["base"] + g)
    u = uniforms(seed, TAG_PARAMS, 2)
    scale = 8 + int(np.floor(9 * u[0]))
    ef = (4, 8, 16, 32)[int(np.floor(4 * u[1]))]
    return scale, ef, seed


def serve_graph_params(g: int):
    """(scale, edge_factor, seed) of resident graph g of the serving set."""
    return 12 + (g % 11), 16, splitmix64(SERVE["base"] + g)


def serve_queries(count: int, n_graphs: int = SERVE["count"], rate: float = SERVE["rate"],
                  mix=SERVE["mix"], seed: int = SERVE["stream_seed"]):
    """Open-loop Poisson query stream.

    Returns arrays: arrival time (s), kind (0 = TC, 1 = BFS, 2 = BC), graph
    id and a per-query seed (used to draw that query's sources)."""
    u = uniforms(seed, TAG_QUERIES, 4 * count).reshape(count, 4)
    gaps = -np.log1p(-u[:, 0]) / rate
    t = np.cumsum(gaps)
    c0, c1 = mix[0], mix[0] + mix[1]
    kind = np.where(u[:, 1] < c0, 0, np.where(u[:, 1] < c1, 1, 2)).astype(np.int32)
    graph = np.minimum((u[:, 2] * n_graphs).astype(np.int64), n_graphs - 1).astype(np.int32)
    qseed = (u[:, 3] * (1 << 53)).astype(np.int64)
    return t, kind, graph, qseed
