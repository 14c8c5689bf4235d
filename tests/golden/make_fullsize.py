"""Writes fullsize_totals.json: exact k-clique totals of the full-size workloads, counted
by the CPU oracle alone (Chiba-Nishizeki recursion, OpenMP over roots): the R-MAT scale-20
graph (k = 3, 4), the Chung-Lu graph with planted communities (k = 6, 7, 8) and, per
graph, the batch of 256 graphs of uneven size (k = 4, 5).  Run from the repository root:
python tests/golden/make_fullsize.py [c2 c3 c4]  (several minutes); named jobs replace
their entries in the existing file."""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_10047_amd import graphgen as gg  # noqa: E402

JOBS = {"c2": (3, 4), "c3": (6, 7, 8)}
BATCH_KS = (4, 5)


def batch_job(threads):
    t = time.time()
    gs = gg.batch_mix(256)
    e = {"graphs": len(gs), "n": [g.n for g in gs], "m": [g.m for g in gs], "totals": {}}
    for k in BATCH_KS:
        e["totals"][str(k)] = [oracle.count(g, k, nthreads=threads) for g in gs]
        print(f"c4 k={k}: sum {sum(e['totals'][str(k)])} ({time.time() - t:.0f}s)", flush=True)
    return e


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_totals.json")
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    names = sys.argv[1:] or ["c2", "c3", "c4"]
    threads = min(16, os.cpu_count() or 1)
    if "c4" in names:
        out["c4"] = batch_job(threads)
    for name, ks in JOBS.items():
        if name not in names:
            continue
        t = time.time()
        g = gg.config_graph(name)
        e = {"n": g.n, "m": g.m, "totals": {}}
        for k in ks:
            t1 = time.time()
            e["totals"][str(k)] = oracle.count(g, k, nthreads=threads)
            print(f"{name} k={k}: {e['totals'][str(k)]} ({time.time() - t1:.0f}s)", flush=True)
        out[name] = e
        print(f"{name}: n={g.n} m={g.m} in {time.time() - t:.0f}s", flush=True)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
