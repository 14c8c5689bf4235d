"""Writes fullsize_totals.json: exact k-clique totals of the full-size workloads, counted
by the CPU oracle alone.  Run from the repository root:
    python tests/golden/make_fullsize.py [c2 c2k5 c3 c4 c5b]
(minutes to an hour per job); named jobs replace their entries in the existing file.

  c2    R-MAT scale 20 (2^24 samples, seed 2), k = 3, 4: Chiba-Nishizeki recursion
  c2k5  the same graph, k = 5: sum over roots of the 4-cliques inside N+(v) on the
        oracle's own peel orientation (the oracle's second counting routine)
  c3    Chung-Lu 2^22 with planted communities (seed 3), k = 6, 7, 8: Chiba-Nishizeki
  c4    the 256-graph batch, per graph, k = 4, 5: Chiba-Nishizeki
  c5b   3-D torus random geometric graph, 2^24 vertices, mean degree 40, seed 52, from
        the counter-based stream (built on the host exactly as on the GPU), k = 5, 6, 7
        by local cliques; with the SHA-256 of its CSR so that the GPU test can show it
        generated the same graph
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2002_10047_amd import graphgen as gg  # noqa: E402

JOBS = {"c2": (3, 4), "c3": (6, 7, 8)}
BATCH_KS = (4, 5)


def csr_digest(offsets, indices) -> str:
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(offsets, np.int64).tobytes())
    h.update(np.ascontiguousarray(indices, np.int32).tobytes())
    return h.hexdigest()


def batch_job(threads):
    t = time.time()
    gs = gg.batch_mix(256)
    e = {"graphs": len(gs), "n": [g.n for g in gs], "m": [g.m for g in gs], "totals": {}}
    for k in BATCH_KS:
        e["totals"][str(k)] = [oracle.count(g, k, nthreads=threads) for g in gs]
        print(f"c4 k={k}: sum {sum(e['totals'][str(k)])} ({time.time() - t:.0f}s)", flush=True)
    return e


def local_totals(g, ks, threads):
    """T_k = sum over roots v of the (k-1)-cliques of G[N+(v)], on the oracle's peel
    orientation, for every k in ks."""
    t = time.time()
    o = oracle.orient(g, 1.0)
    print(f"  oracle orientation {time.time() - t:.0f}s", flush=True)
    jmax = max(ks) - 1
    tot = np.zeros(jmax, dtype=object)
    step = 1 << 20
    for r0 in range(0, g.n, step):
        lc = oracle.local_cliques_roots(g.n, o["ooff"], o["oidx"], jmax, np.arange(r0, min(g.n, r0 + step)),
                                        nthreads=threads)
        tot += np.array([int(x) for x in lc.sum(axis=0, dtype=np.uint64)], dtype=object)
        print(f"  roots < {min(g.n, r0 + step)}: {time.time() - t:.0f}s", flush=True)
    return {str(k): int(tot[k - 2]) for k in ks}


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "fullsize_totals.json")
    names = sys.argv[1:] or ["c2", "c3", "c4"]
    threads = int(os.environ.get("ORACLE_THREADS", min(16, os.cpu_count() or 1)))
    results = {}
    if "c4" in names:
        results["c4"] = batch_job(threads)
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
        results[name] = e
        print(f"{name}: n={g.n} m={g.m} in {time.time() - t:.0f}s", flush=True)
    if "c2k5" in names:
        t = time.time()
        g = gg.config_graph("c2")
        tk = local_totals(g, (5,), threads)
        results["c2k5"] = {"n": g.n, "m": g.m, "totals": tk}
        print(f"c2 k=5: {tk} ({time.time() - t:.0f}s)", flush=True)
    if "c5b" in names:
        t = time.time()
        g = gg.rgg_cb_host(1 << 24, 40.0, seed=52)
        print(f"c5b generated: n={g.n} m={g.m} ({time.time() - t:.0f}s)", flush=True)
        e = {"n": g.n, "m": g.m, "sha256": csr_digest(g.offsets, g.indices),
             "generator": "rgg_cb(n=2^24, dim=3, deg=40, seed=52)"}
        e["totals"] = local_totals(g, (5, 6, 7), threads)
        results["c5b"] = e
        print(f"c5b: {e['totals']} ({time.time() - t:.0f}s)", flush=True)
    out = {}
    if os.path.exists(path):
        with open(path) as f:
            out = json.load(f)
    out.update(results)
    with open(path, "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
