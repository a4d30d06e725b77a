"""Parity of the generic C-ABI operations (mxm, vxm, eWise, assign, reduce)
with the dense GraphBLAS-semantics oracle, over every semiring, mask
variant, accumulator, replace flag and transpose, plus the paper's
Algorithms 1, 3 and 6 written with these calls."""
import itertools

import numpy as np
import pytest
import torch

import graphgen
import oracle
from oracle import semantics as S
from gpu_util import ctx, device_graph, lagr

pytestmark = pytest.mark.gpu

KIND = {"bool": 0, "int64": 1, "fp64": 2, "int32": 3}
NAME = {0: "bool", 1: "int64", 2: "fp64", 3: "int32"}
TDTYPE = {"int64": torch.int64, "fp64": torch.float64, "int32": torch.int32}
SEMIRINGS = {0: "plus.pair", 1: "any.secondi", 2: "plus.first", 3: "min.plus"}
BINOPS = {0: None, 1: "plus", 2: "min", 3: "first", 4: "second", 5: "times", 6: "div", 7: "any"}


def rand_mat(rng, m, n, density, kind):
    e = {}
    for i in range(m):
        for j in range(n):
            if rng.random() < density:
                if kind == "bool":
                    e[(i, j)] = 1
                elif kind == "int64":
                    e[(i, j)] = int(rng.integers(-2, 6))
                elif kind == "int32":
                    # large magnitudes, so that sums and products wrap
                    e[(i, j)] = int(rng.integers(-2 ** 31, 2 ** 31))
                else:
                    e[(i, j)] = float(rng.integers(-2, 6))
    return S.Mat(m, n, e, kind)


def rand_vec(rng, n, density, kind):
    M = rand_mat(rng, 1, n, density, kind)
    return S.Vec(n, {j: v for (_, j), v in M.e.items()}, kind)


def to_dev(M: S.Mat):
    L = lagr()
    keys = sorted(M.e)
    rp = np.zeros(M.nrows + 1, dtype=np.int64)
    for i, _ in keys:
        rp[i + 1] += 1
    rp = np.cumsum(rp)
    ci = np.array([j for _, j in keys], dtype=np.int32)
    vals = None
    if M.kind != "bool":
        vals = torch.tensor([M.e[k] for k in keys], dtype=TDTYPE[M.kind], device="cuda")
    return L.Matrix.wrap_csr(ctx(), M.nrows, M.ncols, torch.from_numpy(rp).cuda(),
                             torch.from_numpy(ci).cuda(), vals, typ=KIND[M.kind])


def from_dev(Mx) -> S.Mat:
    typ, nrows, ncols, nvals = Mx.info()
    rp, ci, va = Mx.to_csr(ctx())
    rp, ci = rp.cpu().numpy(), ci.cpu().numpy()
    va = None if va is None else va.cpu().numpy()
    e = {}
    for i in range(nrows):
        for p in range(rp[i], rp[i + 1]):
            e[(i, int(ci[p]))] = 1 if va is None else va[p].item()
    return S.Mat(nrows, ncols, e, NAME[typ])


def vec_to_dev(v: S.Vec, fmt):
    L = lagr()
    c = ctx()
    idx = sorted(v.e)
    dt = TDTYPE.get(v.kind)
    if fmt == "sparse":
        vals = None if v.kind == "bool" else torch.tensor([v.e[i] for i in idx], dtype=dt, device="cuda")
        return L.Vector.wrap_sparse(c, v.n, torch.tensor(idx, dtype=torch.int32, device="cuda"), vals,
                                    typ=KIND[v.kind])
    pres = torch.zeros(v.n, dtype=torch.uint8)
    pres[idx] = 1
    vals = None
    if v.kind != "bool":
        vals = torch.zeros(v.n, dtype=dt)
        for i in idx:
            vals[i] = v.e[i]
        vals = vals.cuda()
    if fmt == "full" and len(idx) == v.n and v.kind != "bool":
        return L.Vector.wrap_full(c, vals)
    return L.Vector.wrap_bitmap(c, pres.cuda(), vals, typ=KIND[v.kind])


def vec_from_dev(vx) -> S.Vec:
    typ, n, _ = vx.info()
    idx, vals = vx.to_tuples(ctx())
    idx = idx.cpu().numpy()
    vals = None if vals is None else vals.cpu().numpy()
    return S.Vec(n, {int(i): (1 if vals is None else vals[q].item()) for q, i in enumerate(idx)},
                 NAME[typ])


def same(got: dict, want: dict):
    assert set(got) == set(want), (sorted(set(got) ^ set(want)))[:10]
    for k in want:
        assert S.matches(got[k], want[k]), (k, got[k], want[k])


def desc_bits(comp, struct, replace, t0, t1):
    L = lagr()
    return ((L.DESC_COMP if comp else 0) | (L.DESC_STRUCT if struct else 0) |
            (L.DESC_REPLACE if replace else 0) | (L.DESC_TRAN0 if t0 else 0) | (L.DESC_TRAN1 if t1 else 0))


def kinds_for(sr):
    # (A kind, B kind, C kind)
    return {0: ("bool", "int64", "int64"), 1: ("int64", "bool", "int64"),
            2: ("fp64", "bool", "fp64"), 3: ("int64", "fp64", "fp64")}[sr]


@pytest.mark.parametrize("sr", [0, 1, 2, 3])
def test_mxm_all_descriptor_combinations(sr):
    L = lagr()
    rng = np.random.default_rng(100 + sr)
    ak, bk, ck = kinds_for(sr)
    accums = [0, 1, 2, 4]
    for mask_mode, comp, replace, accum, (t0, t1) in itertools.product(
            ("none", "valued", "struct"), (False, True), (False, True), accums,
            ((False, False), (True, False), (False, True), (True, True))):
        m, k, n = 5, 6, 7
        A = rand_mat(rng, k if t0 else m, m if t0 else k, 0.45, ak)
        B = rand_mat(rng, n if t1 else k, k if t1 else n, 0.45, bk)
        C0 = rand_mat(rng, m, n, 0.3, ck)
        M = None if mask_mode == "none" else rand_mat(rng, m, n, 0.5, "int64")
        want = S.mxm(C0, M, BINOPS[accum], SEMIRINGS[sr], A, B, comp=comp,
                     struct=mask_mode == "struct", replace=replace, tran0=t0, tran1=t1,
                     deterministic=True)
        Cd = to_dev(C0)
        Md = None if M is None else to_dev(M)
        L.lagr_mxm(Cd, Md, accum, sr, to_dev(A), to_dev(B),
                   desc_bits(comp, mask_mode == "struct", replace, t0, t1), ctx())
        same(from_dev(Cd).e, want.e)


@pytest.mark.parametrize("fmt_u,fmt_w,fmt_m", [("sparse", "sparse", "sparse"), ("bitmap", "bitmap", "bitmap"),
                                               ("sparse", "full", "bitmap"), ("bitmap", "sparse", "full"),
                                               ("full", "bitmap", "sparse")])
def test_vxm_formats_and_descriptors(fmt_u, fmt_w, fmt_m):
    L = lagr()
    rng = np.random.default_rng(7)
    for sr in range(4):
        ak, bk, ck = kinds_for(sr)
        for comp, struct, replace, t1, accum in itertools.product((False, True), (False, True),
                                                                  (False, True), (False, True), (0, 1)):
            m, n = 8, 9
            u = rand_vec(rng, m, 0.5, ak)
            A = rand_mat(rng, n if t1 else m, m if t1 else n, 0.4, bk)
            w0 = rand_vec(rng, n, 1.0 if fmt_w == "full" else 0.4, ck)
            mk = rand_vec(rng, n, 1.0 if fmt_m == "full" else 0.5, "int64")
            want = S.vxm(w0, mk, BINOPS[accum], SEMIRINGS[sr], u, A, comp=comp, struct=struct,
                         replace=replace, tran1=t1, deterministic=True)
            wd = vec_to_dev(w0, fmt_w)
            L.lagr_vxm(wd, vec_to_dev(mk, fmt_m), accum, sr, vec_to_dev(u, fmt_u), to_dev(A),
                       desc_bits(comp, struct, replace, False, t1), ctx())
            same(vec_from_dev(wd).e, want.e)


@pytest.mark.parametrize("fmt_u", ["sparse", "bitmap", "full"])
@pytest.mark.parametrize("fmt_m", ["sparse", "bitmap", "full"])
def test_vxm_any_secondi_with_parent_assignment(fmt_u, fmt_m):
    """The BFS-shaped call w<!s(p), r> = u any.secondi A' with the parents
    assigned into the mask (p<s(w)> = w), push and pull, on every operand
    format and on sizes past one 256-wide block: w and p against the
    semantics oracle's vxm then assign, and both entry counts (kept on the
    device) against theirs."""
    L = lagr()
    c = ctx()
    rng = np.random.default_rng(31)
    for t1, n, dens in itertools.product((False, True), (9, 700), (0.1, 0.6)):
        u = rand_vec(rng, n, 1.0 if fmt_u == "full" else dens, "int64")
        A = rand_mat(rng, n, n, 4.0 / n, "bool")
        p0 = rand_vec(rng, n, 1.0 if fmt_m == "full" else 0.3, "int64")
        want_w = S.vxm(S.Vec(n, {}, "int64"), p0, None, "any.secondi", u, A, comp=True, struct=True,
                       replace=True, tran1=t1, deterministic=True)
        want_p = S.assign_vector(p0, want_w, None, want_w, struct=True)
        w = L.Vector.new(c, L.INT64, n)
        pd = vec_to_dev(p0, fmt_m)
        L.lagr_vxm(w, pd, 0, L.ANY_SECONDI, vec_to_dev(u, fmt_u), to_dev(A),
                   L.DESC_RSC | L.DESC_ASSIGN_PARENT | (L.DESC_TRAN1 if t1 else 0), c)
        same(vec_from_dev(w).e, want_w.e)
        same(vec_from_dev(pd).e, want_p.e)
        assert w.nvals(c) == len(want_w.e) and pd.nvals(c) == len(want_p.e)


def test_vxm_bfs_loop_allocates_nothing_after_its_first_steps():
    """Algorithm 1's loop on the BFS-shaped fast path: results double-buffer
    through the context, so from the third step on no device memory is
    allocated, and the entry counts are read from the device words."""
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(12, 8, 5)
    G = device_graph(n, s, d)
    A = G.matrix()
    rp, ci = oracle.build_adjacency(n, s, d)
    src = int(graphgen.sources(n, s, d, 1, 5)[0])
    lv, _ = oracle.bfs(rp, ci, src)
    idx = torch.tensor([src], dtype=torch.int32, device="cuda")
    val = torch.tensor([src], dtype=torch.int64, device="cuda")
    q = L.Vector.wrap_sparse(c, n, idx, val, typ=L.INT64)
    p = L.Vector.wrap_sparse(c, n, idx.clone(), val.clone(), typ=L.INT64)
    counts, before = [], None
    for step in range(int(lv.max()) + 1):
        if step == 2:
            before = L.alloc_calls
        L.lagr_vxm(q, p, 0, L.ANY_SECONDI, q, A, L.DESC_RSC | L.DESC_ASSIGN_PARENT, c)
        counts.append(q.nvals(c))
    assert L.alloc_calls == before
    assert counts == [int((lv == k).sum()) for k in range(1, int(lv.max()) + 2)]
    assert p.nvals(c) == int((lv >= 0).sum())


def test_vxm_push_splits_long_rows():
    """Rows longer than the push kernel's batch limit (2,048 entries) are
    walked in chunks by the whole grid: a star with 7,000 leaves plus a
    path, searched with Algorithm 1 from a leaf and from the path's end,
    push and pull, against the queue BFS's smallest parents."""
    from gpu_util import bfs_graphblas
    c = ctx()
    leaves = 7000
    n = leaves + 1 + 50
    edges = [(0, i) for i in range(1, leaves + 1)] + [(leaves + k, leaves + k + 1) for k in range(50)]
    src = np.array([e[0] for e in edges], dtype=np.int32)
    dst = np.array([e[1] for e in edges], dtype=np.int32)
    G = device_graph(n, src, dst)
    rp, ci = oracle.build_adjacency(n, src, dst)
    A = G.matrix()
    for s0 in (3, n - 1):
        lv, _ = oracle.bfs(rp, ci, s0)
        mp = oracle.bfs_min_parent(rp, ci, s0, lv)
        for mode in ("push", "auto"):
            pa, depth = bfs_graphblas(c, A, A, n, s0, mode)
            assert np.array_equal(pa, mp) and depth == int(lv.max())


def test_int32_domain_against_the_semantics_oracle():
    """LAGR_INT32 end to end: wraps widen the caller's int32 values,
    extracts narrow them, and results whose type is INT32 (plus.first over
    an INT32 A, eWise, accumulators, reductions, assign) are taken modulo
    2^32, equal to the semantics oracle's int32 domain; the values are
    drawn over the whole int32 range so that nearly every sum wraps."""
    L = lagr()
    c = ctx()
    rng = np.random.default_rng(41)
    for trial in range(6):
        A = rand_mat(rng, 5, 6, 0.6, "int32")
        B = rand_mat(rng, 6, 7, 0.6, "bool")
        C0 = rand_mat(rng, 5, 7, 0.4, "int32")
        M = rand_mat(rng, 5, 7, 0.6, "int64")
        for accum, comp in ((0, False), (1, False), (2, True), (5, False)):
            want = S.mxm(C0, M, BINOPS[accum], "plus.first", A, B, comp=comp, deterministic=True)
            Cd = to_dev(C0)
            L.lagr_mxm(Cd, to_dev(M), accum, L.PLUS_FIRST, to_dev(A), to_dev(B),
                       desc_bits(comp, False, False, False, False), c)
            same(from_dev(Cd).e, want.e)
        X = rand_mat(rng, 5, 7, 0.5, "int32")
        for op, f in ((1, S.ewise_add), (5, S.ewise_mult), (2, S.ewise_add)):
            want = f(C0, None, BINOPS[1], BINOPS[op], C0, X)
            Cd = to_dev(C0)
            fn = L.lagr_ewise_add if f is S.ewise_add else L.lagr_ewise_mult
            fn(Cd, None, 1, op, to_dev(C0), to_dev(X), 0, c)
            same(from_dev(Cd).e, want.e)
        assert L.lagr_reduce_scalar(to_dev(X), L.PLUS, c) == S.reduce_scalar(X, "plus")
        assert L.lagr_reduce_scalar(to_dev(X), L.MIN, c) == S.reduce_scalar(X, "min")
        w0 = rand_vec(rng, 5, 0.5, "int32")
        for fmt in ("sparse", "bitmap"):
            wd = vec_to_dev(w0, fmt)
            L.lagr_reduce_rows(wd, None, 1, L.PLUS, to_dev(X), 0, c)
            same(vec_from_dev(wd).e, S.reduce_rows(w0, None, "plus", "plus", X).e)
            wd = vec_to_dev(w0, fmt)
            L.lagr_assign_scalar(wd, None, 1, 2 ** 31 - 1, 0, c)
            same(vec_from_dev(wd).e, S.assign_scalar(w0, None, "plus", 2 ** 31 - 1).e)
        u = rand_vec(rng, 5, 1.0, "int32")
        ud = vec_to_dev(u, "full")
        pres, vals = ud.to_dense(c, fill=-3)
        assert vals.dtype == torch.int32 and vals.cpu().tolist() == [u.e[i] for i in range(5)]
        w = L.Vector.new(c, L.INT32, 6)
        L.lagr_vxm(w, None, 0, L.PLUS_FIRST, ud, to_dev(A), 0, c)
        same(vec_from_dev(w).e, S.vxm(S.Vec(6, {}, "int32"), None, None, "plus.first", u, A).e)


@pytest.mark.parametrize("kind", ["fp64", "int64", "bool", "int32"])
def test_plus_first_under_a_complemented_mask_on_lanes(kind):
    """C<!s(M), r> = F plus.first B' with F of at most 64 rows (Algorithm
    3's forward step, one source per row) runs on the lane kernels: against
    the semantics oracle for 1, 5 and 64 rows, both transposes of B, with
    replace and into an empty C; a non-empty C without replace keeps the
    general path and is checked too."""
    L = lagr()
    c = ctx()
    rng = np.random.default_rng(53)
    for ns, n, t1 in itertools.product((1, 5, 64), (300, 700), (False, True)):
        F = rand_mat(rng, ns, n, 0.08, kind)
        B = rand_mat(rng, n, n, 6.0 / n, "bool")
        M = rand_mat(rng, ns, n, 0.3, "int64")
        ck = "int64" if kind == "bool" else kind
        for replace, C0 in ((True, rand_mat(rng, ns, n, 0.1, ck)), (False, S.Mat(ns, n, {}, ck)),
                            (False, rand_mat(rng, ns, n, 0.1, ck))):
            want = S.mxm(C0, M, None, "plus.first", F, B, comp=True, struct=True, replace=replace, tran1=t1)
            Cd = to_dev(C0)
            L.lagr_mxm(Cd, to_dev(M), 0, L.PLUS_FIRST, to_dev(F), to_dev(B),
                       desc_bits(True, True, replace, False, t1), c)
            got = from_dev(Cd).e
            assert set(got) == set(want.e)
            for key, v in want.e.items():
                assert got[key] == v, key           # ascending-k sums on both sides


def test_ewise_assign_reduce():
    L = lagr()
    rng = np.random.default_rng(11)
    for op, accum, mask, comp, replace in itertools.product((1, 2, 3, 4, 5), (0, 1), (False, True),
                                                            (False, True), (False, True)):
        A = rand_mat(rng, 6, 7, 0.5, "int64")
        B = rand_mat(rng, 6, 7, 0.5, "int64")
        C0 = rand_mat(rng, 6, 7, 0.3, "int64")
        M = rand_mat(rng, 6, 7, 0.5, "int64") if mask else None
        for uni in (True, False):
            f = S.ewise_add if uni else S.ewise_mult
            want = f(C0, M, BINOPS[accum], BINOPS[op], A, B, comp=comp, replace=replace)
            Cd = to_dev(C0)
            (L.lagr_ewise_add if uni else L.lagr_ewise_mult)(
                Cd, None if M is None else to_dev(M), accum, op, to_dev(A), to_dev(B),
                desc_bits(comp, False, replace, False, False), ctx())
            same(from_dev(Cd).e, want.e)
    for accum, comp, struct, replace in itertools.product((0, 1, 2), (False, True), (False, True),
                                                          (False, True)):
        w0 = rand_vec(rng, 10, 0.5, "int64")
        u = rand_vec(rng, 10, 0.5, "int64")
        m = rand_vec(rng, 10, 0.5, "int64")
        want = S.assign_vector(w0, m, BINOPS[accum], u, comp=comp, struct=struct, replace=replace)
        wd = vec_to_dev(w0, "sparse")
        L.lagr_assign_vector(wd, vec_to_dev(m, "bitmap"), accum, vec_to_dev(u, "sparse"),
                             desc_bits(comp, struct, replace, False, False), ctx())
        same(vec_from_dev(wd).e, want.e)
        want = S.assign_scalar(w0, m, BINOPS[accum], 7, comp=comp, struct=struct, replace=replace)
        wd = vec_to_dev(w0, "bitmap")
        L.lagr_assign_scalar(wd, vec_to_dev(m, "sparse"), accum, 7,
                             desc_bits(comp, struct, replace, False, False), ctx())
        same(vec_from_dev(wd).e, want.e)
    for kind, monoid, t0 in itertools.product(("int64", "fp64"), (1, 2), (False, True)):
        A = rand_mat(rng, 7, 5, 0.4, kind)
        w0 = S.Vec(5 if t0 else 7, {}, kind)
        want = S.reduce_rows(w0, None, None, BINOPS[monoid], A, tran0=t0)
        wd = vec_to_dev(w0, "sparse")
        L.lagr_reduce_rows(wd, None, 0, monoid, to_dev(A), L.DESC_TRAN0 if t0 else 0, ctx())
        same(vec_from_dev(wd).e, want.e)
        got = L.lagr_reduce_scalar(to_dev(A), monoid, ctx(), fp64=kind == "fp64")
        assert got == S.reduce_scalar(A, BINOPS[monoid])
    empty = S.Mat(3, 3, {}, "int64")
    assert L.lagr_reduce_scalar(to_dev(empty), 1, ctx()) is None


def test_aliased_output():
    L = lagr()
    rng = np.random.default_rng(3)
    A = rand_mat(rng, 6, 6, 0.5, "int64")
    B = rand_mat(rng, 6, 6, 0.5, "int64")
    want = S.mxm(A, A, "plus", "plus.first", A, B, struct=True)
    Ad = to_dev(A)
    L.lagr_mxm(Ad, Ad, 1, 2, Ad, to_dev(B), L.DESC_S, ctx())
    same(from_dev(Ad).e, want.e)


def test_masked_dot_is_per_entry_triangle_counts():
    """C<s(L)> = L plus.pair L^T through lagr_mxm, entry by entry, and the
    fused lagr_mxm_reduce, against the oracle on the 2^10-vertex graph."""
    L = lagr()
    n, s, d = graphgen.rmat_edges(10, 16, 1)
    G = device_graph(n, s, d)
    Lm = L.lagr_select_tril(G.matrix(), ctx())
    C = L.Matrix.new(ctx(), L.INT64, n, n)
    L.lagr_mxm(C, Lm, 0, L.PLUS_PAIR, Lm, Lm, L.DESC_S | L.DESC_TRAN1, ctx())
    rp, ci = oracle.build_adjacency(n, s, d)
    lrp, lci, cnt = oracle.lower_counts(rp, ci)
    rows = np.repeat(np.arange(n), np.diff(lrp))
    want = {(int(i), int(j)): int(c) for i, j, c in zip(rows, lci, cnt) if c > 0}
    assert from_dev(C).e == want
    t = oracle.triangle_count(rp, ci)
    assert L.lagr_mxm_reduce(Lm, L.PLUS_PAIR, Lm, Lm, L.DESC_S | L.DESC_TRAN1, ctx()) == t
    assert L.lagr_reduce_scalar(C, L.PLUS, ctx()) == t
    # the unfused route of mxm_reduce: no transpose flag, so B^T = L^T is
    # formed explicitly and C is built before the reduction (L plus.pair L
    # under s(L) counts each triangle once as well)
    assert L.lagr_mxm_reduce(Lm, L.PLUS_PAIR, Lm, Lm, L.DESC_S, ctx()) == t


def test_min_plus_matches_bellman_ford():
    L = lagr()
    rng = np.random.default_rng(5)
    n = 40
    W = rand_mat(rng, n, n, 0.1, "fp64")
    W = S.Mat(n, n, {k: abs(v) + 1.0 for k, v in W.e.items() if k[0] != k[1]}, "fp64")
    t = S.Vec(n, {0: 0.0}, "fp64")
    td = vec_to_dev(t, "sparse")
    Wd = to_dev(W)
    for _ in range(8):
        t = S.vxm(t, None, "min", "min.plus", t, W)
        L.lagr_vxm(td, None, L.MIN, L.MIN_PLUS, td, Wd, 0, ctx())
        same(vec_from_dev(td).e, t.e)


def test_algorithm1_with_vxm_assign_parent():
    """Algorithm 1 through the C ABI: q<!s(p), r> = q any.secondi A with
    the fused parent assignment; levels equal the queue BFS."""
    L = lagr()
    n, s, d = graphgen.rmat_edges(9, 8, 21)
    rp, ci = oracle.build_adjacency(n, s, d)
    A = S.Mat(n, n, {(i, int(j)): 1 for i in range(n) for j in ci[rp[i]:rp[i + 1]]}, "bool")
    Ad = to_dev(A)
    src = int(graphgen.sources(n, s, d, 1, 21)[0])
    p = vec_to_dev(S.Vec(n, {src: src}, "int64"), "sparse")
    q = vec_to_dev(S.Vec(n, {src: src}, "int64"), "sparse")
    level = {src: 0}
    for lev in range(1, n):
        L.lagr_vxm(q, p, 0, L.ANY_SECONDI, q, Ad, L.DESC_RSC | L.DESC_ASSIGN_PARENT, ctx())
        got = vec_from_dev(q).e
        if not got:
            break
        for v in got:
            level[v] = lev
    lv, _ = oracle.bfs(rp, ci, src)
    assert level == {v: int(lv[v]) for v in range(n) if lv[v] >= 0}
    par = vec_from_dev(p).e
    mp = oracle.bfs_min_parent(rp, ci, src, lv)
    assert par == {v: int(mp[v]) for v in range(n) if lv[v] >= 0}


def test_algorithm3_with_generic_calls():
    """Algorithm 3 (batched Brandes) written with lagr_mxm / eWise / reduce
    on CSR matrices, the backtrack read as i = d down to 1."""
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(8, 8, 33)
    rp, ci = oracle.build_adjacency(n, s, d)
    A = to_dev(S.Mat(n, n, {(i, int(j)): 1 for i in range(n) for j in ci[rp[i]:rp[i + 1]]}, "bool"))
    srcs = [int(x) for x in graphgen.sources(n, s, d, 6, 33)]
    ns = len(srcs)
    P = to_dev(S.Mat(ns, n, {(k, v): 1.0 for k, v in enumerate(srcs)}, "fp64"))
    F = L.Matrix.new(c, L.FP64, ns, n)
    L.lagr_mxm(F, P, 0, L.PLUS_FIRST, P, A, L.DESC_COMP | L.DESC_STRUCT, c)
    Sd = []
    while True:
        Sk = L.Matrix.new(c, L.FP64, ns, n)
        L.lagr_ewise_add(Sk, None, 0, L.PLUS, F, F, 0, c)   # pattern of F
        Sd.append(Sk)
        L.lagr_ewise_add(P, None, 0, L.PLUS, P, F, 0, c)
        L.lagr_mxm(F, P, 0, L.PLUS_FIRST, F, A, L.DESC_RSC, c)
        if F.info()[3] == 0:
            break
    dd = len(Sd) - 1
    B = to_dev(S.Mat(ns, n, {(k, j): 1.0 for k in range(ns) for j in range(n)}, "fp64"))
    W = L.Matrix.new(c, L.FP64, ns, n)
    for i in range(dd, 0, -1):
        L.lagr_ewise_mult(W, Sd[i], 0, L.DIV, B, P, L.DESC_S | L.DESC_REPLACE, c)
        L.lagr_mxm(W, Sd[i - 1], 0, L.PLUS_FIRST, W, A, L.DESC_S | L.DESC_REPLACE | L.DESC_TRAN1, c)
        L.lagr_ewise_mult(B, None, L.PLUS, L.TIMES, W, P, 0, c)
    cent = vec_to_dev(S.Vec(n, {j: -float(ns) for j in range(n)}, "fp64"), "full")
    L.lagr_reduce_rows(cent, None, L.PLUS, L.PLUS, B, L.DESC_TRAN0, c)
    got = np.zeros(n)
    for j, v in vec_from_dev(cent).e.items():
        got[j] = v
    assert np.allclose(got, oracle.brandes(rp, ci, srcs), rtol=1e-12, atol=1e-9)


def test_fp64_valued_mask_treats_both_zeros_as_false():
    """A valued FP64 mask entry is true when present and nonzero (Section
    III, "Masks"): +0.0 and -0.0 both mask the position out, NaN and other
    values keep it.  Checked for mxm (dot and saxpy forms), vxm and assign."""
    L = lagr()
    rng = np.random.default_rng(19)
    m, k, n = 4, 5, 6
    A = rand_mat(rng, m, k, 0.7, "bool")
    B = rand_mat(rng, k, n, 0.7, "int64")
    vals = [0.0, -0.0, 1.5, -2.0, float("nan")]
    M = S.Mat(m, n, {(i, j): vals[(i * n + j) % len(vals)] for i in range(m) for j in range(n)
                     if (i + j) % 3 != 2}, "fp64")
    for comp, replace in itertools.product((False, True), (False, True)):
        C0 = rand_mat(rng, m, n, 0.4, "int64")
        want = S.mxm(C0, M, None, "plus.pair", A, B, comp=comp, replace=replace, deterministic=True)
        Cd = to_dev(C0)
        L.lagr_mxm(Cd, to_dev(M), 0, L.PLUS_PAIR, to_dev(A), to_dev(B),
                   desc_bits(comp, False, replace, False, False), ctx())
        same(from_dev(Cd).e, want.e)
    u = rand_vec(rng, k, 0.8, "bool")
    mk = S.Vec(n, {j: vals[j % len(vals)] for j in range(n)}, "fp64")
    for comp in (False, True):
        w0 = rand_vec(rng, n, 0.4, "int64")
        want = S.vxm(w0, mk, None, "plus.pair", u, B, comp=comp, deterministic=True)
        wd = vec_to_dev(w0, "sparse")
        L.lagr_vxm(wd, vec_to_dev(mk, "sparse"), 0, L.PLUS_PAIR, vec_to_dev(u, "sparse"), to_dev(B),
                   desc_bits(comp, False, False, False, False), ctx())
        same(vec_from_dev(wd).e, want.e)
        w1 = rand_vec(rng, n, 0.5, "int64")
        want = S.assign_scalar(w1, mk, None, 3, comp=comp)
        wd = vec_to_dev(w1, "bitmap")
        L.lagr_assign_scalar(wd, vec_to_dev(mk, "bitmap"), 0, 3, desc_bits(comp, False, False, False, False),
                             ctx())
        same(vec_from_dev(wd).e, want.e)
