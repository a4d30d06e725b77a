"""Parity at the full sizes of the seeded workloads, through the C ABI.

* R-MAT 2^20, ef 16 (seed 2): direction-optimising BFS from all 64 bench
  sources, levels and default (smallest) parents bit for bit against the
  FIFO-queue BFS and the min-parent oracle (Section IV-A, Algorithms 1-2).
  The same search written with lagr_vxm (push only, and push / pull by the
  direction test) from 8 of the sources: parents bit for bit.
* R-MAT 2^18, ef 16 (seed 3): betweenness over the 4 batches of 64 sources,
  summed, against Brandes' FP64 oracle at 1e-12 relative with exact zeros
  (Section IV-B, Algorithm 3).
* The 2,000-graph batch (scales 8-16, edge factors 4-32): every graph's
  triangle count from the one batched launch against a stored file that
  tests/golden/make_golden.py --many writes by calling only the oracle
  (Algorithm 6).
* R-MAT 2^14: the masked per-entry plus.pair product C<s(L)> = L plus.pair
  L' entry by entry (Algorithm 6), and min.plus through lagr_vxm and lagr_mxm
  (Table II; Algorithm 5's semiring): Bellman-Ford rounds to the fixpoint
  against Dijkstra bit for bit, and masked / complement-masked products of
  one-hot rows, which reduce to rows of A.

The oracle side runs in a thread pool: its C calls release the GIL.
"""
import concurrent.futures as cf
import json
import os

import numpy as np
import pytest
import torch

import graphgen
import oracle
from gpu_util import assert_bc_close, bfs_graphblas, ctx, device_graph, lagr

pytestmark = pytest.mark.gpu

POOL = min(16, os.cpu_count() or 4)
GOLD_MANY = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "many_graph_counts.json")


def bfs_host(G, s, flags=0):
    L = lagr()
    c = ctx()
    lv, pv = L.lagr_bfs(G, s, c, flags)
    return lv.values_full(c).cpu().numpy(), pv.values_full(c).cpu().numpy()


def test_bfs_all_64_sources_of_the_2_20_graph():
    cfg = graphgen.LARGE
    n, s, d = graphgen.rmat_edges(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = [int(x) for x in graphgen.sources(n, s, d, cfg["bfs_sources"], cfg["seed"])]
    assert len(srcs) == 64

    def ref(src):
        lv, _ = oracle.bfs(rp, ci, src)
        return lv, oracle.bfs_min_parent(rp, ci, src, lv)

    with cf.ThreadPoolExecutor(POOL) as ex:
        futs = [ex.submit(ref, x) for x in srcs]
        for k, (src, f) in enumerate(zip(srcs, futs)):
            lv, pa = bfs_host(G, src)
            lv_o, mp = f.result()
            futs[k] = None
            assert np.array_equal(lv, lv_o.astype(np.int64)), f"levels differ, source {src}"
            assert np.array_equal(pa, mp), f"parents differ, source {src}"


def test_bfs_written_with_vxm_on_the_2_20_graph():
    L = lagr()
    c = ctx()
    cfg = graphgen.LARGE
    n, s, d = graphgen.rmat_edges(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = [int(x) for x in graphgen.sources(n, s, d, cfg["bfs_sources"], cfg["seed"])][:8]
    A = G.matrix()
    for src in srcs:
        lv, _ = oracle.bfs(rp, ci, src)
        mp = oracle.bfs_min_parent(rp, ci, src, lv)
        for mode in ("push", "auto"):
            pa, depth = bfs_graphblas(c, A, A, n, src, mode)
            assert np.array_equal(pa, mp), f"parents differ, source {src}, {mode}"
            assert depth == int(lv.max())


def test_bc_4_batches_of_64_sources_of_the_2_18_graph():
    L = lagr()
    cfg = graphgen.BC
    n, s, d = graphgen.rmat_edges(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    bs = cfg["batch_size"]
    srcs = graphgen.sources(n, s, d, cfg["batches"] * bs, cfg["seed"])
    assert len(set(int(x) for x in srcs)) == 256
    with cf.ThreadPoolExecutor(cfg["batches"]) as ex:
        parts = list(ex.map(lambda b: oracle.brandes(rp, ci, srcs[b * bs:(b + 1) * bs]),
                            range(cfg["batches"])))
    want = parts[0].copy()
    for p in parts[1:]:
        want += p          # the batches summed in order
    c = ctx()
    got = L.lagr_bc(G, srcs, c).values_full(c).cpu().numpy()
    assert_bc_close(got, want)
    # each batch alone as well
    for b in range(cfg["batches"]):
        gb = L.lagr_bc(G, srcs[b * bs:(b + 1) * bs], c).values_full(c).cpu().numpy()
        assert_bc_close(gb, parts[b])
    # the backward sweep with push levels (chosen per level, and on every level)
    for flags in (L.BC_BACKWARD_PUSH_PULL, L.BC_BACKWARD_PUSH_ONLY):
        assert_bc_close(L.lagr_bc(G, srcs, c, flags).values_full(c).cpu().numpy(), want)


def test_many_graph_batch_counts_equal_the_stored_oracle_counts():
    L = lagr()
    c = ctx()
    with open(GOLD_MANY) as f:
        gold = json.load(f)
    rows = gold["graphs"]
    assert len(rows) == graphgen.MANY["count"]
    gs = []
    for g, scale, ef, nnz, _ in rows:
        assert graphgen.many_graph_params(g)[:2] == (scale, ef)
        n, s, d = graphgen.rmat_edges(*graphgen.many_graph_params(g))
        sd = torch.from_numpy(s).cuda()
        dd = torch.from_numpy(d).cuda()
        A = L.Matrix.build(c, n, n, sd, dd, L.BUILD_SYMMETRIZE | L.BUILD_DROP_LOOPS)
        GG = L.Graph(c, A)
        assert GG.matrix().info()[3] == nnz, f"graph {g}: entries differ from the oracle build"
        L.lagr_property_tc_lower(GG, c)
        gs.append(GG)
    B = L.Batch(c, gs)
    want = np.array([r[4] for r in rows], dtype=np.int64)
    got = B.tc(c, L.Tune(8, 8, 0))
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, f"{bad.size} graphs differ, first {bad[:5].tolist()}"
    tune = B.autotune(c)
    got = B.tc(c)                       # the captured launch, replayed
    assert np.array_equal(got, want), tune.as_dict()
    got = B.tc(c)
    assert np.array_equal(got, want)


def test_per_entry_masked_plus_pair_at_2_14():
    """C<s(L)> = L plus.pair L' through lagr_mxm (DESC_S | TRAN1) on the
    strictly lower part of an R-MAT 2^14 graph, entry by entry against the
    oracle's per-entry intersections, and its reduction."""
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(14, 16, 103)
    G = device_graph(n, s, d)
    Lm = L.lagr_select_tril(G.matrix(), c)
    C = L.Matrix.new(c, L.INT64, n, n)
    L.lagr_mxm(C, Lm, 0, L.PLUS_PAIR, Lm, Lm, L.DESC_S | L.DESC_TRAN1, c)
    rp, ci = oracle.build_adjacency(n, s, d)
    lrp, lci, cnt = oracle.lower_counts(rp, ci)
    keep = cnt > 0
    rows = np.repeat(np.arange(n), np.diff(lrp))
    grp, gci, gva = (t.cpu().numpy() for t in C.to_csr(c))
    grows = np.repeat(np.arange(n), np.diff(grp))
    assert np.array_equal(grows, rows[keep])
    assert np.array_equal(gci, lci[keep])
    assert np.array_equal(gva, cnt[keep])
    assert L.lagr_reduce_scalar(C, L.PLUS, c) == oracle.triangle_count(rp, ci)


def weighted_2_14():
    n, s, d = graphgen.rmat_edges(14, 16, 103)
    rp, ci = oracle.build_adjacency(n, s, d)
    w = graphgen.edge_weights(rp, ci, 140, 255)
    return n, s, d, rp, ci, w


def test_min_plus_vxm_bellman_ford_to_fixpoint_at_2_14():
    """t = t min.plus A with the min accumulator, repeated until t stops
    changing, equals Dijkstra's distances bit for bit (integer weights
    1..255, exact in FP64)."""
    L = lagr()
    c = ctx()
    n, s, d, rp, ci, w = weighted_2_14()
    Wd = L.Matrix.wrap_csr(c, n, n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                           torch.from_numpy(w).cuda())
    for src in graphgen.sources(n, s, d, 3, 140):
        src = int(src)
        want = oracle.dijkstra(rp, ci, w, src)
        t = L.Vector.wrap_sparse(c, n, torch.tensor([src], dtype=torch.int32, device="cuda"),
                                 torch.tensor([0.0], dtype=torch.float64, device="cuda"))
        prev = None
        rounds = 0
        while True:
            L.lagr_vxm(t, None, L.MIN, L.MIN_PLUS, t, Wd, 0, c)
            rounds += 1
            idx, vals = (x.cpu().numpy() for x in t.to_tuples(c))
            cur = (idx.tobytes(), vals.tobytes())
            if cur == prev:
                break
            prev = cur
            assert rounds <= n
        got = np.full(n, np.inf)
        got[idx] = vals
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), src


@pytest.mark.parametrize("comp", [False, True])
def test_min_plus_mxm_one_hot_rows_under_a_mask_at_2_14(comp):
    """C<M> = U min.plus A, U(r, s_r) = x_r one-hot: row r of C is row s_r of
    A plus x_r, kept where the structural mask (or its complement) allows."""
    L = lagr()
    c = ctx()
    n, s, d, rp, ci, w = weighted_2_14()
    Wd = L.Matrix.wrap_csr(c, n, n, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda(),
                           torch.from_numpy(w).cuda())
    rng = np.random.default_rng(1400 + comp)
    k = 48
    rows_src = graphgen.sources(n, s, d, k, 141)
    x = rng.integers(0, 1000, size=k).astype(np.float64) * 0.5
    U = L.Matrix.wrap_csr(c, k, n, torch.arange(k + 1, dtype=torch.int64, device="cuda"),
                          torch.from_numpy(rows_src.astype(np.int32)).cuda(),
                          torch.from_numpy(x).cuda())
    # mask: about a third of each row's candidate columns plus random others
    mrows = []
    for r in range(k):
        cand = ci[rp[rows_src[r]]:rp[rows_src[r] + 1]]
        pick = cand[rng.random(cand.size) < 0.35]
        other = rng.integers(0, n, size=20).astype(np.int32)
        mrows.append(np.unique(np.concatenate([pick, other])))
    mrp = np.zeros(k + 1, dtype=np.int64)
    mrp[1:] = np.cumsum([m.size for m in mrows])
    mci = np.concatenate(mrows).astype(np.int32)
    M = L.Matrix.wrap_csr(c, k, n, torch.from_numpy(mrp).cuda(), torch.from_numpy(mci).cuda(), None,
                          typ=L.BOOL)
    C = L.Matrix.new(c, L.FP64, k, n)
    L.lagr_mxm(C, M, 0, L.MIN_PLUS, U, Wd, L.DESC_S | (L.DESC_COMP if comp else 0), c)
    grp, gci, gva = (t.cpu().numpy() for t in C.to_csr(c))
    for r in range(k):
        u = rows_src[r]
        cols = ci[rp[u]:rp[u + 1]]
        vals = w[rp[u]:rp[u + 1]] + x[r]
        inm = np.isin(cols, mrows[r])
        keep = ~inm if comp else inm
        assert np.array_equal(gci[grp[r]:grp[r + 1]], cols[keep]), r
        assert np.array_equal(gva[grp[r]:grp[r + 1]], vals[keep]), r


def test_batched_bfs_levels_of_all_64_sources_of_the_2_20_graph():
    """lagr_bfs_batch: the 64 bench sources in one multi-source search,
    every (source, vertex) level against the queue BFS."""
    L = lagr()
    c = ctx()
    cfg = graphgen.LARGE
    n, s, d = graphgen.rmat_edges(cfg["scale"], cfg["edge_factor"], cfg["seed"])
    G = device_graph(n, s, d)
    rp, ci = oracle.build_adjacency(n, s, d)
    srcs = [int(x) for x in graphgen.sources(n, s, d, cfg["bfs_sources"], cfg["seed"])]
    lev, reached, lsum, depth = L.lagr_bfs_batch(G, srcs, c)
    with cf.ThreadPoolExecutor(POOL) as ex:
        refs = list(ex.map(lambda x: oracle.bfs(rp, ci, x)[0], srcs))
    for k, (src, ref) in enumerate(zip(srcs, refs)):
        got = lev[k].cpu().numpy()
        assert np.array_equal(got, ref), f"levels differ, source {src}"
        r = ref >= 0
        assert (reached[k], lsum[k], depth[k]) == (int(r.sum()), int(ref[r].sum()), int(ref.max()))
