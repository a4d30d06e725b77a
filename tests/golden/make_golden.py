"""Write tests/golden/oracle_values.json from the seeded inputs and the CPU
oracle only.  Run from the repository root:

    python tests/golden/make_golden.py [--large] [--many]

The paper prints no worked numeric example, so every stored value here is
the oracle's result on a seeded synthetic graph; the oracle itself is pinned
by closed forms and brute force in tests/test_oracle_pins.py.  --large adds
the 2^20-vertex triangle count (minutes of single-threaded CPU time).
--many writes tests/golden/many_graph_counts.json: the triangle count of
every graph of the 2,000-graph batch (scales 8-16, edge factors 4-32), one
oracle call per graph spread over worker processes.
"""
import hashlib
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_values.json")
MANY_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "many_graph_counts.json")

GRAPHS = [(10, 16, 1), (8, 4, 101), (12, 8, 102), (14, 16, 103), (16, 4, 104)]


def csr_sha(rp, ci):
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(rp, dtype=np.int64).tobytes())
    h.update(np.ascontiguousarray(ci, dtype=np.int32).tobytes())
    return h.hexdigest()


def graph_entry(scale, ef, seed, with_bfs_bc):
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    rp, ci = oracle.build_adjacency(n, s, d)
    e = dict(scale=scale, edge_factor=ef, seed=seed, n=n, nnz=int(ci.size),
             sha256=csr_sha(rp, ci), triangles=oracle.triangle_count(rp, ci))
    if with_bfs_bc:
        srcs = graphgen.sources(n, s, d, 8, seed)
        e["sources"] = [int(x) for x in srcs]
        e["bfs_level_sha256"] = []
        for x in srcs:
            lv, _ = oracle.bfs(rp, ci, int(x))
            e["bfs_level_sha256"].append(hashlib.sha256(lv.astype(np.int32).tobytes()).hexdigest())
        bc = oracle.brandes(rp, ci, srcs)
        e["bc_sum"] = float(bc.sum())
        e["bc_max"] = float(bc.max())
    return e


def many_entry(g):
    scale, ef, seed = graphgen.many_graph_params(g)
    n, s, d = graphgen.rmat_edges(scale, ef, seed)
    rp, ci = oracle.build_adjacency(n, s, d)
    return [g, scale, ef, int(ci.size), oracle.triangle_count(rp, ci)]


def write_many():
    import multiprocessing as mp
    count = graphgen.MANY["count"]
    # largest graphs first so the pool ends evenly
    order = sorted(range(count), key=lambda g: -graphgen.many_graph_params(g)[0] * 64
                   - graphgen.many_graph_params(g)[1])
    with mp.Pool(min(16, os.cpu_count() or 4)) as pool:
        rows = sorted(pool.map(many_entry, order, chunksize=1))
    out = {"workload": graphgen.MANY["name"],
           "generator": "graphgen R-MAT a=.57 b=.19 c=.19, SplitMix64 counter-based",
           "columns": ["graph", "scale", "edge_factor", "entries", "triangles"],
           "graphs": rows}
    with open(MANY_OUT, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print("wrote", MANY_OUT)


def main():
    if "--many" in sys.argv:
        write_many()
        return
    large = "--large" in sys.argv
    prev = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            prev = json.load(f)
    out = {"generator": "graphgen R-MAT a=.57 b=.19 c=.19, SplitMix64 counter-based",
           "graphs": [graph_entry(s, ef, sd, s <= 12) for s, ef, sd in GRAPHS]}
    if large:
        out["large"] = graph_entry(20, 16, 2, False)
    elif "large" in prev:
        out["large"] = prev["large"]
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
