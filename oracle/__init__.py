"""CPU oracle for the k-clique counting path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  It shares no code with the HIP library
(``paper_2002_10047_amd``): the C part lives in ``arb_oracle.c`` and is loaded here
with ctypes; the MLP reference is numpy float64 (``oracle.mlp``).

Functions follow the paper (Shi, Dhulipala, Shun, arXiv 2002.10047):
  validate        Sec. 2 (simple undirected graphs)
  orient          Sec. 3.1 and Alg. 4 (peel rounds), Sec. 3.1 last paragraph (directing)
  count           the k-clique definition of Sec. 2, via Chiba-Nishizeki (Sec. 3.4)
  brute           the definition itself, every k-subset tested
  degeneracy      exact degeneracy, for the out-degree bound of Sec. 3.1
  local_cliques   c_j(v), the j-cliques of G[N+(v)] (the per-root work of Alg. 1)
  local_cliques_roots  the same for listed roots (sampled checks at full size)
  vertex_cliques  k-cliques containing listed vertices, from each one's neighbourhood
  approx_peel     arb-approx-peel (Sec. 4.2), rounds of per-vertex counts on the present set
  peel            arb-peel (Alg. 2): remove the least-count vertices, recount, repeat
  features        the per-root scheduling features (d+, sum of d+ over N+, round)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "arb_oracle.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile arb_oracle.c into liboracle.so (gcc, OpenMP, no FP contraction)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        build(force=True)
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.orc_validate.argtypes = [i64, P, P]
    lib.orc_validate.restype = i32
    lib.orc_orient.argtypes = [i64, P, P, dbl, P, P, P, P, P, P, i32]
    lib.orc_orient.restype = i32
    lib.orc_count.argtypes = [i64, P, P, i32, P, i32, i64, i64, P]
    lib.orc_count.restype = ctypes.c_uint64
    lib.orc_brute.argtypes = [i64, P, P, i32, P]
    lib.orc_brute.restype = ctypes.c_uint64
    lib.orc_degeneracy.argtypes = [i64, P, P]
    lib.orc_degeneracy.restype = i64
    lib.orc_local_cliques.argtypes = [i64, P, P, i32, P]
    lib.orc_local_cliques.restype = None
    lib.orc_local_cliques_roots.argtypes = [i64, P, P, i32, P, i64, i32, P]
    lib.orc_local_cliques_roots.restype = None
    lib.orc_vertex_cliques.argtypes = [i64, P, P, i32, P, i64, i32, P]
    lib.orc_vertex_cliques.restype = None
    lib.orc_orient_method.argtypes = [i64, P, P, i32, dbl, P, P, P, P, P, P, i32]
    lib.orc_orient_method.restype = i32
    lib.orc_sparsify.argtypes = [i64, P, P, P, P, P]
    lib.orc_sparsify.restype = i64
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(g):
    off = np.ascontiguousarray(g.offsets, dtype=np.int64)
    idx = np.ascontiguousarray(g.indices, dtype=np.int32)
    if idx.shape[0] == 0:
        idx = np.zeros(1, dtype=np.int32)
    return off, idx


def validate(g) -> int:
    """0 if g is simple, symmetric and sorted; otherwise a nonzero reason code
    (1 offsets, 2 range, 3 self-loop, 4 unsorted/duplicate, 5 asymmetric)."""
    off, idx = _csr(g)
    return int(_load().orc_validate(g.n, _ptr(off), _ptr(idx)))


ORIENT_PEEL, ORIENT_DEGREE, ORIENT_GOODRICH_PSZONA, ORIENT_KCORE = range(4)


def orient(g, eps: float = 1.0, max_rounds: int = 4096, method: int = ORIENT_PEEL):
    """Orientation by the peel (method 0) or by the degree (1), Goodrich-Pszona (2) or
    k-core (3) ordering.  Returns dict with round, deg_at_peel, rank (int32[n]),
    ooff (int64[n+1]), oidx (int32[m]) in rank space, thresholds (int64[rounds])."""
    off, idx = _csr(g)
    n = g.n
    if method == ORIENT_KCORE:
        max_rounds = max(max_rounds, n + 1)
    rnd = np.zeros(max(n, 1), np.int32)
    dap = np.zeros(max(n, 1), np.int32)
    rank = np.zeros(max(n, 1), np.int32)
    ooff = np.zeros(n + 1, np.int64)
    oidx = np.zeros(max(g.m, 1), np.int32)
    thr = np.zeros(max_rounds, np.int64)
    r = _load().orc_orient_method(n, _ptr(off), _ptr(idx), int(method), float(eps), _ptr(rnd), _ptr(dap),
                                  _ptr(rank), _ptr(ooff), _ptr(oidx), _ptr(thr), max_rounds)
    if r < 0:
        raise RuntimeError("orientation exceeded max_rounds")
    return dict(round=rnd[:n], deg_at_peel=dap[:n], rank=rank[:n], ooff=ooff,
                oidx=oidx[:g.m], thresholds=thr[:r], rounds=r)


def count(g, k: int, per_vertex: bool = False, nthreads: int = 1, stride: int = 1, phase: int = 0):
    """Exact number of k-cliques (uint64) and optionally per-vertex incidence counts.
    Raises OverflowError if the total reaches 2^64."""
    off, idx = _csr(g)
    pv = np.zeros(max(g.n, 1), np.uint64) if per_vertex else None
    ov = ctypes.c_int(0)
    t = _load().orc_count(g.n, _ptr(off), _ptr(idx), int(k), _ptr(pv) if pv is not None else None,
                          int(nthreads), int(stride), int(phase), ctypes.byref(ov))
    if ov.value:
        raise OverflowError("k-clique total reached 2^64")
    if per_vertex:
        return int(t), pv[:g.n]
    return int(t)


def brute(g, k: int):
    """(total, per_vertex) by testing every k-subset; n <= 64."""
    if g.n > 64:
        raise ValueError("brute force needs n <= 64")
    off, idx = _csr(g)
    pv = np.zeros(64, np.uint64)
    t = _load().orc_brute(g.n, _ptr(off), _ptr(idx), int(k), _ptr(pv))
    return int(t), pv[:g.n]


def degeneracy(g) -> int:
    off, idx = _csr(g)
    return int(_load().orc_degeneracy(g.n, _ptr(off), _ptr(idx)))


def local_cliques(n: int, ooff: np.ndarray, oidx: np.ndarray, jmax: int) -> np.ndarray:
    """uint64[n, jmax]: entry (v, j-1) = number of j-cliques in G[N+(v)] of the directed graph."""
    ooff = np.ascontiguousarray(ooff, np.int64)
    oidx = np.ascontiguousarray(oidx, np.int32)
    if oidx.shape[0] == 0:
        oidx = np.zeros(1, np.int32)
    out = np.zeros((max(n, 1), max(jmax, 1)), np.uint64)
    if jmax >= 1:
        _load().orc_local_cliques(n, _ptr(ooff), _ptr(oidx), int(jmax), _ptr(out))
    return out[:n, :jmax]


def local_cliques_roots(n: int, ooff: np.ndarray, oidx: np.ndarray, jmax: int, roots, nthreads: int = 0):
    """uint64[len(roots), jmax]: local_cliques for the listed roots only (parallel over roots)."""
    ooff = np.ascontiguousarray(ooff, np.int64)
    oidx = np.ascontiguousarray(oidx, np.int32)
    if oidx.shape[0] == 0:
        oidx = np.zeros(1, np.int32)
    roots = np.ascontiguousarray(roots, np.int64)
    out = np.zeros((max(roots.shape[0], 1), max(jmax, 1)), np.uint64)
    if jmax >= 1 and roots.shape[0]:
        _load().orc_local_cliques_roots(n, _ptr(ooff), _ptr(oidx), int(jmax), _ptr(roots), roots.shape[0],
                                        int(nthreads), _ptr(out))
    return out[:roots.shape[0], :jmax]


def vertex_cliques(g, k: int, verts, nthreads: int = 0) -> np.ndarray:
    """uint64[len(verts)]: number of k-cliques containing each listed vertex, computed from
    its neighbourhood alone ((k-1)-cliques of G[N(v)])."""
    off, idx = _csr(g)
    verts = np.ascontiguousarray(verts, np.int64)
    out = np.zeros(max(verts.shape[0], 1), np.uint64)
    if verts.shape[0]:
        _load().orc_vertex_cliques(g.n, _ptr(off), _ptr(idx), int(k), _ptr(verts), verts.shape[0], int(nthreads),
                                   _ptr(out))
    return out[:verts.shape[0]]


def sparsify(g, colors):
    """Colorful sparsification of g with the given colours: a graph object like g."""
    off, idx = _csr(g)
    col = np.ascontiguousarray(colors, np.int32)
    if col.shape[0] == 0:
        col = np.zeros(1, np.int32)
    out_off = np.zeros(g.n + 1, np.int64)
    out_idx = np.zeros(max(idx.shape[0], 1), np.int32)
    nnz = _load().orc_sparsify(g.n, _ptr(off), _ptr(idx), _ptr(col), _ptr(out_off), _ptr(out_idx))
    return type(g)(g.n, out_off, out_idx[:nnz].copy())


def colorful_estimate(count: int, c: int, k: int) -> float:
    """count * c^(k-1): the appendix's unbiased estimator Y = C / p^(k-1), p = 1/c."""
    return float(count) * float(c) ** (k - 1)


def _induced(g, keep):
    """Subgraph of g on the vertices with keep[v] (same ids; the others isolated)."""
    off, idx = _csr(g)
    u = np.repeat(np.arange(g.n), np.diff(off))
    v = idx[: off[-1]].astype(np.int64)
    sel = keep[u] & keep[v]
    deg = np.bincount(u[sel], minlength=g.n)
    noff = np.zeros(g.n + 1, np.int64)
    noff[1:] = np.cumsum(deg)
    return type(g)(g.n, noff, idx[: off[-1]][sel].astype(np.int32).copy())


def approx_peel(g, k: int, eps: float):
    """arb-approx-peel (Sec. 4.2): while vertices remain, count the k-cliques of the
    present set S per vertex, note the density cliques(S)/|S|, and remove every present
    vertex with at most k(1+eps) times that density k-cliques (compared in double as
    (double)c <= ((double)k * (1 + eps) * (double)cliques) / (double)|S|).  Returns
    (best density, rounds, bool mask of the best S)."""
    keep = np.ones(g.n, bool)
    best, best_mask, rounds = -1.0, keep.copy(), 0
    present = g.n
    while present > 0:
        h = _induced(g, keep)
        C, pv = count(h, k, per_vertex=True, nthreads=8)
        density = float(C) / float(present)
        if density > best:
            best, best_mask = density, keep.copy()
        t = (float(k) * (1.0 + eps) * float(C)) / float(present)
        keep = keep & ~(pv.astype(np.float64) <= t)
        present = int(keep.sum())
        rounds += 1
    return max(best, 0.0), rounds, best_mask


def peel(g, k: int):
    """arb-peel (Alg. 2) by definition: while vertices remain, count the k-cliques of the
    present set S per vertex (from scratch), remove every vertex with the least count
    (its round is r), and note the density cliques / |S| of what remains (the whole
    graph first).  Returns (best density, rounds, round per vertex)."""
    keep = np.ones(g.n, bool)
    rnd = -np.ones(g.n, np.int32)
    T = count(g, k, nthreads=8)
    best = float(T) / float(g.n) if g.n else 0.0
    r = 0
    while keep.any():
        h = _induced(g, keep)
        _, pv = count(h, k, per_vertex=True, nthreads=8)
        low = pv[keep].min()
        A = keep & (pv == low)
        rnd[A] = r
        keep = keep & ~A
        r += 1
        if keep.any():
            C = count(_induced(g, keep), k, nthreads=8)
            best = max(best, float(C) / float(keep.sum()))
    return best, r, rnd


def features(n: int, ooff: np.ndarray, oidx: np.ndarray, round_rank_space: np.ndarray) -> np.ndarray:
    """float64[n, 3]: (d+(v), sum over u in N+(v) of d+(u), round(v)) in rank space."""
    dplus = np.diff(np.asarray(ooff, np.int64))
    rows = np.repeat(np.arange(n), dplus)
    s = np.zeros(n, np.float64)
    np.add.at(s, rows, dplus[np.asarray(oidx, np.int64)].astype(np.float64))
    return np.stack([dplus.astype(np.float64), s, np.asarray(round_rank_space, np.float64)], axis=1)
