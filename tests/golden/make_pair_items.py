"""Writes pair_items.json: oracle k-clique totals and per-vertex counts of the two-block
stochastic block model sbm2(2000, 0.05, 0.85, seed 11) at k = 5, 6.  Its 279 roots with
more than 768 out-neighbours are counted through per-out-neighbour (root, child) items at
k >= 5, so these values pin that path.  Counted by the CPU oracle alone (Chiba-Nishizeki
recursion, OpenMP over roots).  Run from the repository root:
python tests/golden/make_pair_items.py  (about a minute)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_10047_amd import graphgen as gg  # noqa: E402

GRAPH = ("sbm2", 2000, 0.05, 0.85, 11)
KS = (5, 6)


def main():
    g = gg.sbm2(*GRAPH[1:])
    out = {"graph": list(GRAPH), "n": g.n, "m": g.m, "totals": {}, "per_vertex": {}}
    for k in KS:
        t, pv = oracle.count(g, k, per_vertex=True, nthreads=min(16, os.cpu_count() or 1))
        out["totals"][str(k)] = t
        out["per_vertex"][str(k)] = [int(x) for x in pv]
        print(f"k={k}: {t}", flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pair_items.json")
    with open(path, "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
