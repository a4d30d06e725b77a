"""Many-graph triangle counting in one (graph-captured) launch against the
oracle, graph by graph, and against the single-graph path."""
import numpy as np
import pytest

import graphgen
import oracle
from gpu_util import ctx, device_graph, lagr, graph_from_edges
import graphs as Gs

pytestmark = pytest.mark.gpu


def small_batch(count, seed0):
    gs, want = [], []
    for g in range(count):
        seed = graphgen.splitmix64(seed0 + g)
        u = graphgen.uniforms(seed, graphgen.TAG_PARAMS, 2)
        scale = 4 + int(8 * u[0])          # 16 .. 2048 vertices
        ef = (1, 4, 8, 16, 32)[int(5 * u[1])]
        n, s, d = graphgen.rmat_edges(scale, ef, seed)
        gs.append(device_graph(n, s, d))
        want.append(oracle.triangle_count(*oracle.build_adjacency(n, s, d)))
    return gs, np.array(want, dtype=np.int64)


def test_batched_counts_equal_oracle_and_replays():
    L = lagr()
    c = ctx()
    gs, want = small_batch(60, 77 << 32)
    # edge cases in the same batch: an empty graph, a triangle, K_40
    for g in (Gs.path(1), Gs.cycle(3), Gs.complete(40)):
        G, (rp, ci) = graph_from_edges(*g)
        gs.append(G)
        want = np.append(want, oracle.triangle_count(rp, ci))
    B = L.Batch(c, gs)
    ng, rows, entries = B.info()
    assert ng == len(gs)
    eager = B.tc(c, L.Tune(4, 2, 0))
    assert np.array_equal(eager, want)
    for t in (L.Tune(1, 1, 0), L.Tune(8, 4, 0), L.Tune(2, 64, 0), L.Tune(16, 2, 0)):
        assert np.array_equal(B.tc(c, t), want)
    # replays of the captured launch, with other device work in between
    graph_tune = L.Tune(8, 2, 1)
    for rep in range(4):
        assert np.array_equal(B.tc(c, graph_tune), want), rep
        assert L.lagr_tc(gs[rep], c) == want[rep]
    best = B.autotune(c)
    assert best.use_graph == 1 and 1 <= best.blocks_per_cu <= 16
    assert np.array_equal(B.tc(c), want)
    assert np.array_equal(B.tc(c), want)


def test_single_graph_batch_and_bad_tune():
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(10, 16, 1)
    G = device_graph(n, s, d)
    B = L.Batch(c, [G])
    assert B.tc(c).tolist() == [oracle.triangle_count(*oracle.build_adjacency(n, s, d))]
    with pytest.raises(L.LagrError) as e:
        B.tc(c, L.Tune(0, 2, 0))
    assert e.value.code == L.INVALID_VALUE
    with pytest.raises(L.LagrError) as e:
        B.tc(c, L.Tune(4, 0, 0))
    assert e.value.code == L.INVALID_VALUE
