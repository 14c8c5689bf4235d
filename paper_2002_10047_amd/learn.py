"""Learned cost model for the counting schedule: data, training and inference driver.

Every numerical step runs in libarb.so kernels (arb_features, the instrumented
arb_count_async, arb_mlp_forward, arb_mse_grad, arb_mlp_backward, arb_adam_step); this
module only sequences them and moves tensors.

The label of a root v is log2(1 + w(v)) where w(v) is the work measure the counting
kernels report for v (gathered out-neighbour words plus bitmap words of its search
tree; its sum over roots is the O(m alpha^(k-2)) work of Alg. 1, Sec. 3.2).  The
features are (log2(1+d+(v)), log2(1 + sum_{u in N+(v)} d+(u)), peel round of v).
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import arb

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
H = 64
SHAPES = [(H, 3), (H,), (H, H), (H,), (H, H), (H,), (1, H), (1,)]


def init_weights(seed: int) -> np.ndarray:
    """He-style initial fp32 weights (biases zero), flat layout of include/arb.h."""
    g = np.random.Generator(np.random.PCG64(seed))
    parts = []
    for s in SHAPES:
        if len(s) == 2:
            parts.append(g.normal(0.0, np.sqrt(2.0 / s[1]), size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def graph_rows(g, k: int, eps: float = 1.0, device="cuda"):
    """(X float32[R,3], y float32[R]) for the roots of g with d+ >= k-1."""
    off, idx = arb.to_device_csr(g, device)
    o = arb.arb_orient(off, idx, eps=eps)
    feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])
    n = g.n
    work = torch.empty(max(n, 1), dtype=torch.int64, device=device)
    arb.arb_count_async(o["ooff"], o["oidx"], k, work=work)
    dplus = (o["ooff"][1:] - o["ooff"][:-1])
    live = dplus >= (k - 1)
    w = work[:n][live].to(torch.float64)
    y = torch.log2(1.0 + w).to(torch.float32)
    return feat[live].contiguous(), y.contiguous()


class Trainer:
    """Adam on fp32 master weights with a bf16 copy used by the kernels."""

    def __init__(self, seed: int = 0, lr: float = 3e-3, device="cuda"):
        self.w = torch.from_numpy(init_weights(seed)).to(device)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.wb = arb.arb_to_bf16(self.w)
        self.lr = lr
        self.step_no = 0

    def step(self, X, y):
        pred, act = arb.arb_mlp_forward(self.wb, X, want_act=True)
        dy, loss = arb.arb_mse_grad(pred, y)
        grad = arb.arb_mlp_backward(self.wb, X, act, dy)
        self.step_no += 1
        arb.arb_adam_step(self.w, self.wb, grad, self.m, self.v, self.lr, self.step_no)
        return loss

    def loss(self, X, y):
        pred = arb.arb_mlp_forward(self.wb, X)
        _, loss = arb.arb_mse_grad(pred, y)
        return float(loss.item())


def train(X, y, steps: int = 3000, batch: int = 4096, lr: float = 3e-3, seed: int = 0, Xval=None, yval=None,
          log_every: int = 500, log=None):
    """Minibatch training; returns (trainer, history of (step, train_loss, val_loss))."""
    tr = Trainer(seed=seed, lr=lr, device=X.device)
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    hist = []
    R = X.shape[0]
    for s in range(1, steps + 1):
        if R > batch:
            sel = torch.randint(0, R, (batch,), device=X.device, generator=gen)
            tr.step(X[sel].contiguous(), y[sel].contiguous())
        else:
            tr.step(X, y)
        if s % log_every == 0 or s == steps:
            tl = tr.loss(X, y)
            vl = tr.loss(Xval, yval) if Xval is not None else float("nan")
            hist.append((s, tl, vl))
            if log:
                log(f"step {s}: train {tl:.4f} val {vl:.4f}")
    return tr, hist


def save_weights(wb: torch.Tensor, k: int, meta: dict, out_dir: str = WEIGHTS_DIR):
    import json
    os.makedirs(out_dir, exist_ok=True)
    bits = wb.cpu().numpy().view(np.uint16)
    np.save(os.path.join(out_dir, f"cost_mlp_k{k}.npy"), bits)
    with open(os.path.join(out_dir, f"cost_mlp_k{k}.json"), "w") as f:
        json.dump(meta, f, indent=1)


def load_weights(k: int, device="cuda"):
    """bf16 weight bits of the cost model for clique size k (int16 device tensor), or None."""
    p = os.path.join(WEIGHTS_DIR, f"cost_mlp_k{k}.npy")
    if not os.path.exists(p):
        return None
    bits = np.load(p).astype(np.uint16)
    return torch.from_numpy(bits.view(np.int16).copy()).to(device)
