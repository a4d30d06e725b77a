"""The query server against the oracle, and the same query set answered in
batches and one query at a time (results must agree bit for bit)."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import ctx, device_graph, lagr, graph_from_edges, assert_bc_close
import graphs as Gs

pytestmark = pytest.mark.gpu


def resident_set():
    """Graphs with long rows (hub chunks), a deep path, a disconnected graph
    and two R-MAT graphs, with their host CSR."""
    gs, csr = [], []
    for scale, ef, seed in ((10, 16, 901), (11, 8, 902)):
        n, s, d = graphgen.rmat_edges(scale, ef, seed)
        gs.append(device_graph(n, s, d))
        csr.append(oracle.build_adjacency(n, s, d))
    for g in (Gs.star(2500), Gs.path(700),
              Gs.disjoint_union(Gs.complete(30), Gs.wheel(600))):
        G, (rp, ci) = graph_from_edges(*g)
        gs.append(G)
        csr.append((rp, ci))
    return gs, csr


def query_set(csr, seed=3):
    """TC, BFS and BC queries over every graph, in a seeded order."""
    L = lagr()
    rng = np.random.default_rng(seed)
    qs = []
    for g, (rp, ci) in enumerate(csr):
        n = rp.size - 1
        qs.append((L.QUERY_TC, g, ()))
        for s in rng.integers(0, n, size=9):
            qs.append((L.QUERY_BFS, g, (int(s),)))
        qs.append((L.QUERY_BFS, g, (0,)))
        qs.append((L.QUERY_BFS, g, (0,)))       # duplicate query
        for k in (1, 3, 8, 8):
            qs.append((L.QUERY_BC, g, tuple(int(x) for x in rng.integers(0, n, size=k))))
    order = rng.permutation(len(qs))
    return [qs[i] for i in order]


def expected(csr, q):
    kind, g, src = q
    rp, ci = csr[g]
    if kind == 0:
        return {"triangles": oracle.triangle_count(rp, ci)}
    if kind == 1:
        lev = oracle.bfs(rp, ci, src[0])[0]
        r = lev >= 0
        return {"reached": int(r.sum()), "level_sum": int(lev[r].sum()), "depth": int(lev.max()),
                "level": lev}
    c = oracle.brandes(rp, ci, np.array(src, dtype=np.int64))
    return {"bc_sum": float(c.sum()), "bc_max": float(c.max()), "bc": c}


def run(server, qs, arrival=0.0):
    L = lagr()
    tickets = [server.submit(L.make_query(k, g, s, arrival)) for k, g, s in qs]
    assert server.wait(len(qs), 120.0), server.stats()
    res = {r.ticket: r for r in server.poll(len(qs) + 16)}
    assert sorted(res) == sorted(tickets)
    return [res[t] for t in tickets], tickets


def check_against_oracle(csr, qs, res):
    for q, r in zip(qs, res):
        assert r.status == 0, (q, r.status)
        want = expected(csr, q)
        if q[0] == 0:
            assert r.triangles == want["triangles"], q
        elif q[0] == 1:
            assert (r.reached, r.level_sum, r.depth) == (want["reached"], want["level_sum"],
                                                         want["depth"]), q
        else:
            assert r.bc_sum == pytest.approx(want["bc_sum"], rel=1e-11, abs=1e-9), q
            assert r.bc_max == pytest.approx(want["bc_max"], rel=1e-12, abs=0), q


FIELDS = ("status", "triangles", "reached", "level_sum", "depth", "bc_sum", "bc_max")


def test_server_batched_equals_oracle_and_alone():
    L = lagr()
    c = ctx()
    gs, csr = resident_set()
    qs = query_set(csr)
    mixed = L.Server(c, gs, workers=2, keep_vectors=True)
    res_mixed, t_mixed = run(mixed, qs)
    st = mixed.stats()
    assert st["completed"] == len(qs) and st["rejected"] == 0
    # all queries were visible at once: BFS and BC ran in shared batches
    assert st["batches"][1] < st["queries"][1] and st["batches"][2] < st["queries"][2]
    assert max(r.batch_size for r in res_mixed) > 1
    check_against_oracle(csr, qs, res_mixed)
    vec_mixed = {}
    for q, r, t in zip(qs, res_mixed, t_mixed):
        if q[0] == 0:
            continue
        v = mixed.result_vector(t, c).values_full(c).cpu().numpy()
        want = expected(csr, q)
        if q[0] == 1:
            assert np.array_equal(v, want["level"].astype(np.int64)), q
        else:
            assert_bc_close(v, want["bc"])
        vec_mixed[t] = v
    taken = next(t for q, t in zip(qs, t_mixed) if q[0] != 0)
    with pytest.raises(L.LagrError):
        mixed.result_vector(taken, c)   # each kept vector is handed over once
    mixed.free()

    alone = L.Server(c, gs, workers=1, max_bfs_batch=1, max_bc_batch=1, keep_vectors=True)
    res_alone, t_alone = run(alone, qs)
    assert all(r.batch_size == 1 for r in res_alone if r.kind != 0)
    for q, a, b, ta, tb in zip(qs, res_mixed, res_alone, t_mixed, t_alone):
        for f in FIELDS:
            assert getattr(a, f) == getattr(b, f), (q, f)
        if q[0] != 0:
            v = alone.result_vector(tb, c).values_full(c).cpu().numpy()
            assert np.array_equal(v, vec_mixed[ta]), q
    alone.free()


def test_server_arrival_gating_and_budget():
    L = lagr()
    c = ctx()
    gs, csr = resident_set()
    n_big = max(rp.size - 1 for rp, _ in csr)
    big = int(np.argmax([rp.size - 1 for rp, _ in csr]))
    # a budget that holds any BFS batch but no BC batch of the largest graph
    budget = 200 * n_big
    S = L.Server(c, gs, workers=3, budget_bytes=budget)
    t0 = S.clock()
    qs = [(L.QUERY_BFS, g, (1,)) for g in range(len(gs))]
    qs += [(L.QUERY_TC, g, ()) for g in range(len(gs))]
    qs += [(L.QUERY_BC, big, (0, 1))]
    arrivals = [t0 + 0.2 + 0.01 * i for i in range(len(qs))]
    tickets = [S.submit(L.make_query(k, g, s, a)) for (k, g, s), a in zip(qs, arrivals)]
    assert S.wait(len(qs), 60.0)
    res = {r.ticket: r for r in S.poll()}
    for (k, g, s), t, a in zip(qs, tickets, arrivals):
        r = res[t]
        assert r.arrival == a
        assert r.start >= a and r.done >= r.start
        if k == L.QUERY_BC:
            assert r.status == L.BUDGET_EXCEEDED
        else:
            assert r.status == 0
            want = expected(csr, (k, g, s))
            if k == L.QUERY_TC:
                assert r.triangles == want["triangles"]
            else:
                assert r.reached == want["reached"] and r.depth == want["depth"]
    st = S.stats()
    assert st["rejected"] == 1 and 0 < st["peak_bytes"] <= budget
    # the device's measured use and the accounted use after the stream
    assert st["device_peak_bytes"] > 0 and 0 <= st["held_bytes"]
    S.free()


def test_server_rejects_bad_queries():
    L = lagr()
    c = ctx()
    G, (rp, ci) = graph_from_edges(*Gs.cycle(5))
    S = L.Server(c, [G], workers=1)
    bad = [L.make_query(7, 0, ()), L.make_query(L.QUERY_BFS, 1, (0,)),
           L.make_query(L.QUERY_BFS, 0, (5,)), L.make_query(L.QUERY_BFS, 0, (0, 1)),
           L.make_query(L.QUERY_BC, 0, ()), L.make_query(L.QUERY_TC, 0, (1,))]
    codes = []
    for q in bad:
        with pytest.raises(L.LagrError) as e:
            S.submit(q)
        codes.append(e.value.code)
    assert codes == [-2, -3, -3, -2, -2, -2]
    assert S.stats()["pending"] == 0
    t = S.submit(L.make_query(L.QUERY_TC, 0, ()))
    assert t == 0 and S.wait(1, 30.0)
    assert S.poll()[0].triangles == 0
    S.free()
    with pytest.raises(L.LagrError):
        L.Server(c, [G], workers=0)
