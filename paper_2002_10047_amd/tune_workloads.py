"""Run the autotuner (arb_autotune) on the benchmark workloads and store the options in
the package's cache (tuned/count_opts.json), for the degree and learned schedules.

Workloads: rgg3d (3-D torus RGG, 2^24 vertices, mean degree 40, k = 5, 6, 7), rmat26
(R-MAT scale 26, k = 4), rmat20 (R-MAT scale 20, k = 3, 4, 5), chunglu (Chung-Lu 2^22
with planted communities, k = 6, 7, 8).

Usage: python -m paper_2002_10047_amd.tune_workloads [rgg3d rmat26 rmat20 chunglu] [--trials N] [--cache FILE]
"""
from __future__ import annotations

import argparse
import sys
import time

import torch

from . import arb
from . import graphgen as gg
from . import learn, tuning


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(name):
    if name == "rgg3d":
        n, off, idx = gg.rgg_cb_device(1 << 24, 40.0, seed=52)
        return off, idx, (5, 6, 7)
    if name == "rmat26":
        n, off, idx = gg.rmat_cb_device(26, 1 << 30, seed=51)
        return off, idx, (4,)
    if name == "rmat20":
        off, idx = arb.to_device_csr(gg.config_graph("c2"))
        return off, idx, (3, 4, 5)
    if name == "chunglu":
        off, idx = arb.to_device_csr(gg.config_graph("c3"))
        return off, idx, (6, 7, 8)
    raise KeyError(name)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="*", default=["rgg3d", "rmat26", "rmat20", "chunglu"])
    ap.add_argument("--trials", type=int, default=2)
    ap.add_argument("--schedules", default="degree,learned")
    ap.add_argument("--cache", default=tuning.CACHE, help="options cache to update (default: the package's)")
    a = ap.parse_args()
    for name in a.names:
        t0 = time.time()
        off, idx, ks = workload(name)
        o = arb.arb_orient(off, idx, eps=1.0)
        feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])
        log(f"{name}: n={off.numel() - 1} m={idx.numel() // 2} ready in {time.time() - t0:.1f}s")
        for k in ks:
            ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
            w = learn.load_weights(k)
            for sched in a.schedules.split(","):
                t1 = time.time()
                op, ms = tuning.tuned_opts(o["ooff"], o["oidx"], k, sched, mlp_weights=w if sched == "learned" else None,
                                           features=feat if sched == "learned" else None, ws=ws, retune=True,
                                           trials=a.trials, path=a.cache)
                log(f"{name} k={k} {sched}: {ms:.3f} ms {arb.opts_dict(op)} (search {time.time() - t1:.0f}s)")
            del ws
        del o, feat, off, idx
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main()
