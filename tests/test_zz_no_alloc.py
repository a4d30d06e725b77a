"""The allocation-free triangle count (lagr_tc_adv_noalloc) against
lagr_tc_adv, the entry point it varies: two calls in a row on one fresh
context, the second on a smaller graph, both equal to lagr_tc_adv's count,
and no device allocation made by either call."""
import numpy as np
import pytest
import torch

import graphgen
from gpu_util import ctx, device_graph, lagr

pytestmark = pytest.mark.gpu


def test_noalloc_count_equals_the_allocating_count_twice():
    L = lagr()
    c = ctx()
    graphs = []
    for scale, ef, seed in ((16, 16, 31), (10, 8, 32)):      # the second is smaller
        n, s, d = graphgen.rmat_edges(scale, ef, seed)
        G = device_graph(n, s, d)
        L.lagr_property_tc_lower(G, c)
        graphs.append((G, L.lagr_tc_adv(G, c)))
    assert graphs[0][1] > graphs[1][1] > 0
    fresh = L.Context(0)              # no workspace: any allocation would show
    out = torch.full((2,), -1, dtype=torch.int64, device="cuda")
    before = L.alloc_calls
    for k, (G, want) in enumerate(graphs):
        L.lagr_tc_adv_noalloc(G, out[k:k + 1], fresh)
    fresh.wait()
    assert L.alloc_calls == before, "the allocation-free count allocated"
    assert out.cpu().tolist() == [graphs[0][1], graphs[1][1]]
    # again in the other order on the same scratch (it keeps the last call's
    # counters, which each call clears)
    out.fill_(-1)
    for k, (G, want) in enumerate(reversed(graphs)):
        L.lagr_tc_adv_noalloc(G, out[k:k + 1], fresh)
    fresh.wait()
    assert out.cpu().tolist() == [graphs[1][1], graphs[0][1]]
    fresh.free()


def test_noalloc_count_rejects_an_unprepared_graph():
    L = lagr()
    c = ctx()
    n, s, d = graphgen.rmat_edges(8, 8, 33)
    G = device_graph(n, s, d)
    out = torch.zeros(1, dtype=torch.int64, device="cuda")
    with pytest.raises(L.LagrError) as e:
        L.lagr_tc_adv_noalloc(G, out, c)
    assert e.value.code == L.PROPERTY_MISSING
