"""Train the per-k cost models of the learned schedule and store them in weights/.

Training data: the batch of 256 graphs of uneven size (G(n,p) with mean degree 16,
R-MAT scales 12-18, 2-D random geometric graphs with mean degree 20; 10^4 to 5*10^5
edges, seeds 4000+g).  Graphs g < 192 train, g >= 192 validate.  Every number is
produced by libarb.so kernels: orientation, features, the instrumented count that
measures each root's work, and the MLP forward/backward/Adam steps.

Usage: python -m paper_2002_10047_amd.train_cost [--ks 3,4,5,6] [--steps 4000]
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import graphgen as gg
from . import learn


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def spearman(a, b):
    ra = np.argsort(np.argsort(a)).astype(np.float64)
    rb = np.argsort(np.argsort(b)).astype(np.float64)
    ra -= ra.mean()
    rb -= rb.mean()
    return float((ra * rb).sum() / np.sqrt((ra * ra).sum() * (rb * rb).sum()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--ks", default="3,4,5,6")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--graphs", type=int, default=256)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--out", default=learn.WEIGHTS_DIR)
    a = ap.parse_args()
    t0 = time.time()
    gs = gg.batch_mix(a.graphs)
    ntr = (a.graphs * 3) // 4
    log(f"batch: {len(gs)} graphs, {sum(g.m for g in gs)} edges, generated in {time.time() - t0:.1f}s")
    for k in [int(x) for x in a.ks.split(",")]:
        t1 = time.time()
        rows = [learn.graph_rows(g, k) for g in gs]
        Xtr = torch.cat([r[0] for r in rows[:ntr]])
        ytr = torch.cat([r[1] for r in rows[:ntr]])
        Xva = torch.cat([r[0] for r in rows[ntr:]])
        yva = torch.cat([r[1] for r in rows[ntr:]])
        log(f"k={k}: {Xtr.shape[0]} training roots, {Xva.shape[0]} validation roots ({time.time() - t1:.1f}s)")
        v0 = learn.Trainer(seed=0).loss(Xva, yva)
        tr, hist = learn.train(Xtr, ytr, steps=a.steps, lr=a.lr, Xval=Xva, yval=yva, log_every=500, log=log)
        from . import arb
        pred = arb.arb_mlp_forward(tr.wb, Xva).cpu().numpy()
        yv = yva.cpu().numpy()
        deg = Xva[:, 0].cpu().numpy()
        meta = {
            "k": k, "train_graphs": f"batch_mix g < {ntr} (seeds 4000+g)", "val_graphs": f"g >= {ntr}",
            "train_roots": int(Xtr.shape[0]), "val_roots": int(Xva.shape[0]), "steps": a.steps, "lr": a.lr,
            "batch": 4096, "val_loss_init": v0, "history": hist,
            "val_spearman_model": spearman(pred, yv), "val_spearman_degree": spearman(deg, yv),
            "label": "log2(1 + work), work as reported by the instrumented count",
            "features": "log2(1+d+), log2(1+sum of out-neighbours' d+), peel round",
        }
        log(f"k={k}: val loss {v0:.3f} -> {hist[-1][2]:.4f}; rank correlation model {meta['val_spearman_model']:.4f} "
            f"vs degree {meta['val_spearman_degree']:.4f}")
        learn.save_weights(tr.wb, k, meta, a.out)
    log(f"done in {time.time() - t0:.1f}s")


if __name__ == "__main__":
    main()
