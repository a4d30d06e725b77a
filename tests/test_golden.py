"""Regression of the seeded inputs and the oracle against stored values
written by tests/golden/make_golden.py (oracle-only)."""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_values.json")


def load():
    with open(GOLD) as f:
        return json.load(f)


@pytest.mark.parametrize("entry", load()["graphs"], ids=lambda e: f"s{e['scale']}ef{e['edge_factor']}")
def test_generator_and_oracle_regression(entry):
    n, s, d = graphgen.rmat_edges(entry["scale"], entry["edge_factor"], entry["seed"])
    rp, ci = oracle.build_adjacency(n, s, d)
    h = hashlib.sha256()
    h.update(rp.astype(np.int64).tobytes())
    h.update(ci.astype(np.int32).tobytes())
    assert (n, int(ci.size), h.hexdigest()) == (entry["n"], entry["nnz"], entry["sha256"])
    assert oracle.triangle_count(rp, ci) == entry["triangles"]
    if "sources" in entry:
        srcs = graphgen.sources(n, s, d, 8, entry["seed"])
        assert [int(x) for x in srcs] == entry["sources"]
        for x, want in zip(srcs, entry["bfs_level_sha256"]):
            lv, _ = oracle.bfs(rp, ci, int(x))
            assert hashlib.sha256(lv.astype(np.int32).tobytes()).hexdigest() == want
        bc = oracle.brandes(rp, ci, srcs)
        assert abs(bc.sum() - entry["bc_sum"]) <= 1e-9 * entry["bc_sum"]


def test_small_graph_has_the_expected_magnitude():
    """The 2^10-vertex graph has about 21k stored entries and 7.7e4 triangles."""
    e = load()["graphs"][0]
    assert e["scale"] == 10 and 0.95 * 21150 <= e["nnz"] <= 1.05 * 21150


def test_many_graph_golden_spot_check():
    """A few of the stored 2,000-graph counts (written by make_golden.py
    --many from the oracle) recomputed: the generator and oracle still agree."""
    with open(os.path.join(os.path.dirname(GOLD), "many_graph_counts.json")) as f:
        rows = json.load(f)["graphs"]
    assert len(rows) == graphgen.MANY["count"]
    small = [r for r in rows if r[1] <= 10][:6]
    for g, scale, ef, nnz, tri in small:
        assert graphgen.many_graph_params(g)[:2] == (scale, ef)
        n, s, d = graphgen.rmat_edges(*graphgen.many_graph_params(g))
        rp, ci = oracle.build_adjacency(n, s, d)
        assert (int(ci.size), oracle.triangle_count(rp, ci)) == (nnz, tri)
