"""Write tests/golden/oracle_values.json from the seeded inputs and the CPU
oracle only.  Run from the repository root:

    python tests/golden/make_golden.py [--large]

The paper prints no worked numeric example, so every stored value here is
the oracle's result on a seeded synthetic graph; the oracle itself is pinned
by closed forms and brute force in tests/test_oracle_pins.py.  --large adds
the 2^20-vertex triangle count (minutes of single-threaded CPU time).
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


def main():
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
