"""Float64 reference of the scheduling cost model.  TEST INFRASTRUCTURE ONLY.

The cost model is not from the paper: it predicts the per-root work of Alg. 1 (whose
total the paper bounds in Sec. 3.2) from three per-root features, so that the heaviest
roots are scheduled and split first.  Network: 3 -> 64 -> 64 -> 64 -> 1, ReLU after each
hidden layer, linear output.  Parameters are one flat vector of 8641 values laid out as
W1[64][3] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[1][64] b4[1] (W[out][in]).

The GPU kernels hold the weights in bfloat16 and accumulate in float32; this reference
takes the same bf16-rounded weights and float32 inputs and computes in float64.

Loss: L = sum_r (y_r - t_r)^2 / (2 N); its gradient wrt y_r is (y_r - t_r) / N.
Optimiser: Adam (Kingma & Ba, 2015) with bias correction.
"""
from __future__ import annotations

import numpy as np

H = 64
SHAPES = [("W1", (H, 3)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)),
          ("W3", (H, H)), ("b3", (H,)), ("W4", (1, H)), ("b4", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    p = np.asarray(p, np.float64)
    out, o = {}, 0
    for name, s in SHAPES:
        c = int(np.prod(s))
        out[name] = p[o:o + c].reshape(s)
        o += c
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float64).ravel() for name, _ in SHAPES])


def bf16_round(x):
    """float -> nearest bfloat16 (ties to even), returned as float32 values."""
    u = np.asarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def bf16_bits(x):
    return (bf16_round(x).view(np.uint32) >> 16).astype(np.uint16)


def from_bf16_bits(b):
    return (np.asarray(b, np.uint16).astype(np.uint32) << 16).view(np.float32)


def init_params(seed: int):
    """He-style initialisation (weights ~ N(0, 2/fan_in), biases 0)."""
    g = np.random.Generator(np.random.PCG64(seed))
    d = {}
    for name, s in SHAPES:
        if name.startswith("W"):
            d[name] = g.normal(0.0, np.sqrt(2.0 / s[1]), size=s)
        else:
            d[name] = np.zeros(s)
    return pack(d)


def forward(params, X):
    """Returns (y[N], cache) with cache = (x, z1, h1, z2, h2, z3, h3)."""
    P = unpack(params)
    x = np.asarray(X, np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.maximum(z2, 0.0)
    z3 = h2 @ P["W3"].T + P["b3"]
    h3 = np.maximum(z3, 0.0)
    y = h3 @ P["W4"].T + P["b4"]
    return y[:, 0], (x, z1, h1, z2, h2, z3, h3)


def backward(params, cache, dy):
    """Gradient of sum_r dy_r * y_r wrt the flat parameter vector (chain rule)."""
    P = unpack(params)
    x, z1, h1, z2, h2, z3, h3 = cache
    dy = np.asarray(dy, np.float64)[:, None]
    g = {}
    g["W4"] = dy.T @ h3
    g["b4"] = dy.sum(axis=0)
    d3 = (dy @ P["W4"]) * (z3 > 0)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(axis=0)
    d2 = (d3 @ P["W3"]) * (z2 > 0)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(axis=0)
    d1 = (d2 @ P["W2"]) * (z1 > 0)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(axis=0)
    return pack(g)


def loss_and_dy(y, t):
    y = np.asarray(y, np.float64)
    t = np.asarray(t, np.float64)
    r = y - t
    return float((r * r).sum() / (2 * len(y))), r / len(y)


def adam_step(w, g, m, v, lr, step, b1=0.9, b2=0.999, eps=1e-8):
    """One bias-corrected Adam update; returns new (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
