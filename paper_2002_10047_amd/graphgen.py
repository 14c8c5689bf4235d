"""Seeded synthetic graph generators shared by the tests, the benchmark and the oracle checks.

This module only produces inputs: simple undirected graphs in CSR form (int64 row
offsets, int32 column indices, every row sorted ascending, both directions of each
edge present, no self-loops, no duplicates).  It holds none of the clique-counting
or orientation arithmetic, so neither the HIP path nor the CPU oracle depends on the
other through it.

Randomness comes from numpy's PCG64 generator seeded explicitly (the same seed and
numpy version give the same graph byte for byte), or, for the counter-based families,
from SplitMix64 evaluated at each draw's index on either side.

Workload families (the shapes the paper's experiments use are social/web graphs of
Table 1; these synthetic families stand in for them):

* ``er_planted``   G(n, m) with a planted clique
* ``rmat``         recursive-matrix (R-MAT) power-law graph
* ``chung_lu``     Chung-Lu expected-degree power-law graph with planted dense communities
* ``rgg``          random geometric graph on the unit torus (2-D or 3-D)
* ``rmat_cb_*``, ``rgg_cb_*``  R-MAT and 3-D RGG from a counter-based stream, built
                   identically on the GPU (torch) and on the host (numpy)
* ``batch_mix``    a batch of graphs of uneven size mixing G(n,p), R-MAT and 2-D RGG
* small exact families: complete, Turan, cycle, star, empty, G(n,p)
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "Graph", "rng", "csr_from_pairs", "er_planted", "rmat", "chung_lu", "rgg",
    "batch_mix", "disjoint_union", "complete", "turan", "cycle", "star", "empty",
    "gnp", "gnm", "relabel", "config_graph",
]


@dataclass
class Graph:
    """Undirected simple graph in symmetric CSR form."""
    n: int
    offsets: np.ndarray   # int64[n+1]
    indices: np.ndarray   # int32[2m]
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.indices.shape[0])

    @property
    def m(self) -> int:
        return self.nnz // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.offsets)

    def edges(self):
        """Each undirected edge once as (u, v) with u < v."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.indices.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def csr_from_pairs(n: int, u, v, name: str = "") -> Graph:
    """Drop self-loops and duplicate pairs, then build the symmetric sorted CSR."""
    n = int(n)
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    del u, v, keep
    key = np.unique(lo * n + hi)
    del lo, hi
    lo = key // n
    hi = key - lo * n
    del key
    both = np.empty(2 * lo.shape[0], dtype=np.int64)
    both[: lo.shape[0]] = lo * n + hi
    both[lo.shape[0]:] = hi * n + lo
    del lo, hi
    both.sort(kind="stable")
    src = both // n
    indices = (both - src * n).astype(np.int32)
    del both
    counts = np.bincount(src, minlength=n).astype(np.int64)
    del src
    offsets = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=offsets[1:])
    return Graph(n, offsets, indices, name)


def _distinct_pairs(g: np.random.Generator, n: int, m: int):
    """m distinct uniformly random unordered pairs {a, b}, a != b."""
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("more edges than pairs")
    chosen = np.empty(0, dtype=np.int64)
    while chosen.shape[0] < m:
        need = m - chosen.shape[0]
        a = g.integers(0, n, size=2 * need + 16, dtype=np.int64)
        b = g.integers(0, n, size=2 * need + 16, dtype=np.int64)
        keep = a != b
        key = np.minimum(a, b)[keep] * n + np.maximum(a, b)[keep]
        allk = np.concatenate([chosen, key])
        _, first = np.unique(allk, return_index=True)
        first.sort()
        chosen = allk[first][:m]
    return chosen // n, chosen % n


def gnm(n: int, m: int, seed: int, name: str = "") -> Graph:
    g = rng(seed)
    a, b = _distinct_pairs(g, n, m)
    return csr_from_pairs(n, a, b, name or f"gnm(n={n},m={m},seed={seed})")


def gnp(n: int, p: float, seed: int, name: str = "") -> Graph:
    """Erdos-Renyi G(n, p): every pair independently with probability p."""
    g = rng(seed)
    total = n * (n - 1) // 2
    m = int(g.binomial(total, p)) if total else 0
    a, b = _distinct_pairs(g, n, m) if m else (np.empty(0, np.int64), np.empty(0, np.int64))
    return csr_from_pairs(n, a, b, name or f"gnp(n={n},p={p},seed={seed})")


def sbm2(n: int, p_in: float, p_out: float, seed: int, name: str = "") -> Graph:
    """Two-block stochastic block model: vertices [0, n/2) and [n/2, n); a pair inside a
    block is an edge with probability p_in, a pair across the blocks with p_out.  With
    p_out >> p_in the degrees are high while cliques stay rare (most edges are bipartite)."""
    g = rng(seed)
    h = n // 2
    a0, b0 = np.triu_indices(h, 1)
    keep = g.random(a0.size) < p_in
    keep2 = g.random(a0.size) < p_in
    cross = g.random((h, n - h)) < p_out
    ca, cb = np.nonzero(cross)
    u = np.concatenate([a0[keep], h + a0[keep2], ca]).astype(np.int64)
    v = np.concatenate([b0[keep], h + b0[keep2], h + cb]).astype(np.int64)
    return csr_from_pairs(n, u, v, name or f"sbm2(n={n},p_in={p_in},p_out={p_out},seed={seed})")


def er_planted(n: int = 2000, m: int = 20000, clique: int = 30, seed: int = 1) -> Graph:
    """G(n, m) plus a clique on `clique` distinct uniformly chosen vertices (union, deduped)."""
    g = rng(seed)
    a, b = _distinct_pairs(g, n, m)
    members = g.choice(n, size=clique, replace=False).astype(np.int64)
    ia, ib = np.triu_indices(clique, 1)
    a = np.concatenate([a, members[ia]])
    b = np.concatenate([b, members[ib]])
    gr = csr_from_pairs(n, a, b, f"er_planted(n={n},m={m},K{clique},seed={seed})")
    gr.planted = np.sort(members)
    return gr


def rmat(scale: int, nsamples: int, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2, permute: bool = True, chunk: int = 1 << 23) -> Graph:
    """R-MAT: each sample descends `scale` levels choosing a quadrant with probs a, b, c, d.

    Quadrant a keeps (row, col) bits (0, 0), b gives (0, 1), c gives (1, 0), d gives (1, 1).
    A seeded random vertex permutation is applied, then self-loops and duplicates go.
    """
    g = rng(seed)
    n = 1 << scale
    us, vs = [], []
    left = nsamples
    while left > 0:
        cnt = min(chunk, left)
        left -= cnt
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for lvl in range(scale):
            r = g.random(cnt)
            bit = np.int64(1) << np.int64(scale - 1 - lvl)
            row1 = r >= (a + b)
            col1 = ((r >= a) & (r < a + b)) | (r >= a + b + c)
            u |= row1.astype(np.int64) * bit
            v |= col1.astype(np.int64) * bit
        us.append(u)
        vs.append(v)
    u = np.concatenate(us)
    v = np.concatenate(vs)
    del us, vs
    if permute:
        perm = g.permutation(n).astype(np.int64)
        u = perm[u]
        v = perm[v]
    return csr_from_pairs(n, u, v, f"rmat(scale={scale},samples={nsamples},seed={seed})")


# ---------------------------------------------------------------- counter-based generators
#
# The two largest workloads are generated on the GPU (seconds) and, identically, on the
# host (minutes; for oracle totals).  Both draw from SplitMix64 (Steele, Lea and Flood,
# "Fast splittable pseudorandom number generators", OOPSLA 2014), whose i-th output for
# seed s is mix(s + (i + 1) * GAMMA): every draw is a function of its index alone, so the
# two sides agree draw for draw and chunks can be generated in any order.  A uniform
# double is the top 53 bits times 2^-53 (exact on both sides), and every comparison that
# decides an edge is the same IEEE operations on both sides.

_M64 = (1 << 64) - 1
_SM_GAMMA = 0x9E3779B97F4A7C15
_SM_M1 = 0xBF58476D1CE4E5B9
_SM_M2 = 0x94D049BB133111EB
_STREAM_RMAT, _STREAM_PERM, _STREAM_RGG = 1, 2, 3


def _mix_int(z: int) -> int:
    z &= _M64
    z = ((z ^ (z >> 30)) * _SM_M1) & _M64
    z = ((z ^ (z >> 27)) * _SM_M2) & _M64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    """64-bit key of one stream of draws of a seeded workload."""
    return _mix_int((_mix_int(int(seed)) + int(stream) * _SM_GAMMA) & _M64)


def _signed(x: int) -> int:
    return x - (1 << 64) if x >= (1 << 63) else x


def sm64_np(key: int, i) -> np.ndarray:
    """uint64 SplitMix64 output number i (integer array) of the generator keyed `key`."""
    with np.errstate(over="ignore"):
        z = np.uint64(key) + (np.asarray(i).astype(np.uint64) + np.uint64(1)) * np.uint64(_SM_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_SM_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_SM_M2)
    return z ^ (z >> np.uint64(31))


def _srl_t(z, s: int):
    """logical right shift of an int64 tensor holding uint64 bits"""
    return (z >> s) & ((1 << (64 - s)) - 1)


def sm64_torch(key: int, i):
    """sm64_np on an int64 tensor of indices (any device): int64 tensor of the uint64 bits
    (two's-complement wrap-around of int64 addition and multiplication)."""
    z = (i + 1) * _signed(_SM_GAMMA) + _signed(key)
    z = (z ^ _srl_t(z, 30)) * _signed(_SM_M1)
    z = (z ^ _srl_t(z, 27)) * _signed(_SM_M2)
    return z ^ _srl_t(z, 31)


def unif_np(key: int, i) -> np.ndarray:
    return (sm64_np(key, i) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def unif_torch(key: int, i):
    import torch
    return _srl_t(sm64_torch(key, i), 11).to(torch.float64) * (2.0 ** -53)


def rmat_cb_permutation_np(scale: int, seed: int) -> np.ndarray:
    """The vertex relabelling of the counter-based R-MAT: ids sorted (stably) by a 63-bit
    draw each; vertex u becomes perm[u]."""
    n = 1 << scale
    keys = (sm64_np(stream_key(seed, _STREAM_PERM), np.arange(n, dtype=np.int64)) >> np.uint64(1)).astype(np.int64)
    return np.argsort(keys, kind="stable").astype(np.int64)


def rmat_cb_host(scale: int, nsamples: int, a: float = 0.57, b: float = 0.19, c: float = 0.19, seed: int = 51,
                 chunk: int = 1 << 22) -> "Graph":
    """R-MAT (as rmat()) from the counter-based stream: sample i at level l uses draw
    i * scale + l; ids relabelled by rmat_cb_permutation_np; self-loops and duplicates
    dropped.  Byte-identical to rmat_cb_device(scale, nsamples, seed=seed)."""
    kr = stream_key(seed, _STREAM_RMAT)
    perm = rmat_cb_permutation_np(scale, seed)
    ab, abc = a + b, a + b + c
    keys = []
    for i0 in range(0, nsamples, chunk):
        cnt = min(chunk, nsamples - i0)
        i = np.arange(i0, i0 + cnt, dtype=np.int64) * scale
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for lvl in range(scale):
            r = unif_np(kr, i + lvl)
            bit = np.int64(1) << np.int64(scale - 1 - lvl)
            u |= (r >= ab).astype(np.int64) * bit
            v |= (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64) * bit
        u, v = perm[u], perm[v]
        keep = u != v
        u, v = u[keep], v[keep]
        keys.append(np.unique((np.minimum(u, v) << scale) | np.maximum(u, v)))
    key = np.unique(np.concatenate(keys)) if keys else np.empty(0, np.int64)
    del keys
    off, idx = host_csr_from_keys(key, scale, 1 << scale)
    return Graph(1 << scale, off, idx, f"rmat_cb(scale={scale},samples={nsamples},seed={seed})")


def rmat_cb_device(scale: int, nsamples: int, a: float = 0.57, b: float = 0.19, c: float = 0.19, seed: int = 51,
                   device="cuda", chunk: int = 1 << 24):
    """rmat_cb_host generated on the GPU with torch elementwise operations: (n, offsets
    int64[n+1], indices int32[2m]) device tensors, byte-identical to the host graph."""
    import torch
    n = 1 << scale
    kr = stream_key(seed, _STREAM_RMAT)
    pk = _srl_t(sm64_torch(stream_key(seed, _STREAM_PERM), torch.arange(n, dtype=torch.int64, device=device)), 1)
    perm = torch.sort(pk, stable=True).indices
    del pk
    ab, abc = a + b, a + b + c
    keys = []
    for i0 in range(0, nsamples, chunk):
        cnt = min(chunk, nsamples - i0)
        i = torch.arange(i0, i0 + cnt, dtype=torch.int64, device=device) * scale
        u = torch.zeros(cnt, dtype=torch.int64, device=device)
        v = torch.zeros(cnt, dtype=torch.int64, device=device)
        for lvl in range(scale):
            r = unif_torch(kr, i + lvl)
            bit = 1 << (scale - 1 - lvl)
            u |= (r >= ab).to(torch.int64) * bit
            v |= (((r >= a) & (r < ab)) | (r >= abc)).to(torch.int64) * bit
        del i, r
        u = perm[u]
        v = perm[v]
        keep = u != v
        u, v = u[keep], v[keep]
        keys.append(torch.unique((torch.minimum(u, v) << scale) | torch.maximum(u, v)))
        del u, v, keep
    key = torch.unique(torch.cat(keys))           # sorted, one entry per undirected edge
    del keys
    off, idx = _device_csr_from_keys(key, scale, n)
    return n, off, idx


def host_csr_from_keys(key: np.ndarray, bits: int, n: int):
    """numpy counterpart of _device_csr_from_keys: sorted unique keys lo << bits | hi
    (lo < hi) -> (offsets int64[n+1], indices int32[2m]), rows ascending."""
    key = np.asarray(key, np.int64)
    m = key.shape[0]
    mask = (1 << bits) - 1
    lo = key >> bits
    hi = key & mask
    deg_up = np.bincount(lo, minlength=n).astype(np.int64)
    deg_dn = np.bincount(hi, minlength=n).astype(np.int64)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(deg_up + deg_dn, out=off[1:])
    idx = np.empty(2 * m, dtype=np.int32)
    first_up = np.cumsum(deg_up) - deg_up
    idx[off[lo] + deg_dn[lo] + (np.arange(m, dtype=np.int64) - first_up[lo])] = hi.astype(np.int32)
    del first_up
    k2 = np.sort((hi << bits) | lo)
    del lo, hi
    hi2 = k2 >> bits
    lo2 = k2 & mask
    del k2
    first_dn = np.cumsum(deg_dn) - deg_dn
    idx[off[hi2] + (np.arange(m, dtype=np.int64) - first_dn[hi2])] = lo2.astype(np.int32)
    return off, idx


def _rgg_radius(n: int, avg_deg: float) -> float:
    return (avg_deg / ((4.0 / 3.0) * math.pi * n)) ** (1.0 / 3.0)


def rgg_cb_host(n: int, avg_deg: float = 40.0, seed: int = 52) -> "Graph":
    """3-D random geometric graph on the unit torus from the counter-based stream (point
    i's coordinate j is draw 3 i + j): an edge iff dx*dx + dy*dy + dz*dz <= r*r, with
    d = min(|a - b|, 1 - |a - b|) per axis, summed left to right, and
    r = (avg_deg / (4/3 pi n))^(1/3).  Candidate pairs come from a k-d tree at a slightly
    larger radius and are decided by that expression, so the graph is byte-identical to
    rgg_cb_device(n, avg_deg, seed)."""
    from scipy.spatial import cKDTree
    pts = unif_np(stream_key(seed, _STREAM_RGG), np.arange(3 * n, dtype=np.int64)).reshape(n, 3)
    r = _rgg_radius(n, avg_deg)
    tree = cKDTree(pts, boxsize=1.0)
    pairs = tree.query_pairs(r * (1.0 + 1e-9), output_type="ndarray")
    del tree
    keep = np.zeros(pairs.shape[0], bool)
    step = 1 << 24
    for s0 in range(0, pairs.shape[0], step):
        a = pts[pairs[s0:s0 + step, 0]]
        b = pts[pairs[s0:s0 + step, 1]]
        dv = np.abs(a - b)
        dv = np.minimum(dv, 1.0 - dv)
        d2 = dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1] + dv[:, 2] * dv[:, 2]
        keep[s0:s0 + step] = d2 <= r * r
    pairs = pairs[keep]
    bits = max(1, (n - 1).bit_length())
    lo = np.minimum(pairs[:, 0], pairs[:, 1]).astype(np.int64)
    hi = np.maximum(pairs[:, 0], pairs[:, 1]).astype(np.int64)
    del pairs
    key = np.unique((lo << bits) | hi)
    del lo, hi
    off, idx = host_csr_from_keys(key, bits, n)
    return Graph(n, off, idx, f"rgg_cb(n={n},dim=3,deg={avg_deg},seed={seed})")


def rgg_cb_device(n: int, avg_deg: float = 40.0, seed: int = 52, device="cuda", chunk: int = 1 << 21):
    """rgg_cb_host built on the GPU with a cell list (cells of side >= r; the 27 cells
    around each point's cell are searched): (n, offsets int64[n+1], indices int32[2m])
    device tensors, byte-identical to the host graph."""
    import torch
    r = _rgg_radius(n, avg_deg)
    G = max(3, int(math.floor(1.0 / r)))            # cells per axis, side 1/G >= r
    pts = unif_torch(stream_key(seed, _STREAM_RGG), torch.arange(3 * n, dtype=torch.int64, device=device)).view(n, 3)
    cxyz = torch.clamp((pts * G).to(torch.int64), max=G - 1)
    cell = (cxyz[:, 0] * G + cxyz[:, 1]) * G + cxyz[:, 2]
    cell_sorted, order = torch.sort(cell)
    ncell = G * G * G
    cstart = torch.zeros(ncell + 1, dtype=torch.int64, device=device)
    cstart[1:] = torch.cumsum(torch.bincount(cell_sorted, minlength=ncell), 0)
    kmax = int((cstart[1:] - cstart[:-1]).max())
    bits = max(1, (n - 1).bit_length())
    r2 = r * r
    keys = []
    for c0 in range(0, n, chunk):
        ids = order[c0:c0 + chunk]                  # points of this chunk, in cell order
        cx, cy, cz = cxyz[ids, 0], cxyz[ids, 1], cxyz[ids, 2]
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    nc = (((cx + dx) % G) * G + (cy + dy) % G) * G + (cz + dz) % G
                    s0 = cstart[nc]
                    cnt = cstart[nc + 1] - s0
                    for t in range(kmax):
                        ok = cnt > t
                        if not bool(ok.any()):
                            break
                        src = ids[ok]
                        dst = order[s0[ok] + t]
                        keep = src < dst
                        src, dst = src[keep], dst[keep]
                        dv = torch.abs(pts[src] - pts[dst])
                        dv = torch.minimum(dv, 1.0 - dv)
                        d2 = dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1] + dv[:, 2] * dv[:, 2]
                        close = d2 <= r2
                        keys.append((src[close] << bits) | dst[close])
    key = torch.unique(torch.cat(keys))
    del keys
    off, idx = _device_csr_from_keys(key, bits, n)
    return n, off, idx


def _device_csr_from_keys(key, bits: int, n: int):
    """CSR (offsets int64[n+1], indices int32[2m]) on key's device from sorted unique keys
    lo << bits | hi, lo < hi: row r lists its neighbours below r, then those above r."""
    import torch
    device = key.device
    lo = key >> bits
    hi = key & ((1 << bits) - 1)
    m = lo.numel()
    deg_up = torch.bincount(lo, minlength=n)      # neighbours above each vertex
    deg_dn = torch.bincount(hi, minlength=n)      # neighbours below
    off = torch.zeros(n + 1, dtype=torch.int64, device=device)
    off[1:] = torch.cumsum(deg_up + deg_dn, 0)
    idx = torch.empty(2 * m, dtype=torch.int32, device=device)
    # row lo, upper part: after its deg_dn lower neighbours, in key order (ascending hi)
    first_up = torch.cumsum(deg_up, 0) - deg_up
    idx[off[lo] + deg_dn[lo] + (torch.arange(m, device=device) - first_up[lo])] = hi.to(torch.int32)
    del first_up
    # row hi, lower part: neighbours lo in ascending order, at the start of the row
    k2, _ = torch.sort((hi << bits) | lo)
    del lo, hi
    hi2 = k2 >> bits
    lo2 = k2 & ((1 << bits) - 1)
    del k2
    first_dn = torch.cumsum(deg_dn, 0) - deg_dn
    idx[off[hi2] + (torch.arange(m, device=device) - first_dn[hi2])] = lo2.to(torch.int32)
    return off, idx


def _capped_weights(n: int, beta: float, total: float, wmax: float) -> np.ndarray:
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (beta - 1.0))
    for _ in range(100):
        w *= total / w.sum()
        over = w > wmax
        if not over.any():
            break
        w[over] = wmax
    return w


def chung_lu(n: int, beta: float, npairs: int, wmax: float, ncomm: int = 0,
             comm_lo: int = 40, comm_hi: int = 80, comm_p: float = 0.5, seed: int = 3,
             chunk: int = 1 << 23) -> Graph:
    """Chung-Lu power-law graph with planted dense communities.

    Weights w_i proportional to (i+1)^(-1/(beta-1)), scaled so that sum(w) = 2*npairs and
    capped at wmax (iterated rescale).  `npairs` endpoint pairs are drawn i.i.d. with each
    endpoint proportional to w.  Then `ncomm` disjoint communities, sizes uniform in
    [comm_lo, comm_hi], each an internal G(s, comm_p), are added.  Ids are permuted.
    """
    g = rng(seed)
    w = _capped_weights(n, beta, 2.0 * npairs, wmax)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    us, vs = [], []
    left = npairs
    while left > 0:
        cnt = min(chunk, left)
        left -= cnt
        us.append(np.minimum(np.searchsorted(cdf, g.random(cnt), side="right"), n - 1))
        vs.append(np.minimum(np.searchsorted(cdf, g.random(cnt), side="right"), n - 1))
    sizes = g.integers(comm_lo, comm_hi + 1, size=ncomm)
    pool = g.permutation(n)
    pos = 0
    for s in sizes:
        mem = pool[pos:pos + s].astype(np.int64)
        pos += s
        ia, ib = np.triu_indices(int(s), 1)
        keep = g.random(ia.shape[0]) < comm_p
        us.append(mem[ia[keep]])
        vs.append(mem[ib[keep]])
    u = np.concatenate(us).astype(np.int64)
    v = np.concatenate(vs).astype(np.int64)
    del us, vs
    perm = g.permutation(n).astype(np.int64)
    return csr_from_pairs(n, perm[u], perm[v],
                          f"chung_lu(n={n},beta={beta},pairs={npairs},wmax={wmax},comm={ncomm},seed={seed})")


def rgg(n: int, dim: int, avg_deg: float, seed: int) -> Graph:
    """Random geometric graph: n uniform points on the unit torus [0,1)^dim, edge iff distance <= r,
    with r chosen so that the expected degree is avg_deg."""
    from scipy.spatial import cKDTree
    g = rng(seed)
    pts = g.random((n, dim))
    if dim == 2:
        r = math.sqrt(avg_deg / (math.pi * n))
    elif dim == 3:
        r = (avg_deg / ((4.0 / 3.0) * math.pi * n)) ** (1.0 / 3.0)
    else:
        raise ValueError("dim must be 2 or 3")
    tree = cKDTree(pts, boxsize=1.0)
    pairs = tree.query_pairs(r, output_type="ndarray")
    return csr_from_pairs(n, pairs[:, 0], pairs[:, 1], f"rgg(n={n},dim={dim},deg={avg_deg},seed={seed})")


def disjoint_union(graphs):
    """Disjoint union of graphs; returns (Graph, vertex_offsets int64[G+1])."""
    vo = np.zeros(len(graphs) + 1, dtype=np.int64)
    eo = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, gr in enumerate(graphs):
        vo[i + 1] = vo[i] + gr.n
        eo[i + 1] = eo[i] + gr.nnz
    offs = np.empty(vo[-1] + 1, dtype=np.int64)
    idx = np.empty(eo[-1], dtype=np.int32)
    for i, gr in enumerate(graphs):
        offs[vo[i]:vo[i + 1]] = gr.offsets[:-1] + eo[i]
        idx[eo[i]:eo[i + 1]] = gr.indices.astype(np.int64) + vo[i]
    offs[-1] = eo[-1]
    return Graph(int(vo[-1]), offs, idx, f"union({len(graphs)})"), vo


def batch_mix(count: int = 256, m_lo: float = 1e4, m_hi: float = 5e5, seed_base: int = 4000,
              scale_m: float = 1.0):
    """Batch of graphs of uneven size.  Graph g uses seed seed_base+g and type g mod 3:
    0 -> G(n,p) with mean degree 16, 1 -> R-MAT (a,b,c)=(.57,.19,.19) with scale
    clamp(round(log2(m/16)),12,18), 2 -> 2-D RGG on the torus with mean degree 20.
    Target edge counts are log-uniform in [m_lo, m_hi] (times scale_m)."""
    out = []
    for gi in range(count):
        g = rng(seed_base + gi)
        mg = int(math.exp(g.uniform(math.log(m_lo), math.log(m_hi))) * scale_m)
        t = gi % 3
        s = seed_base + gi + 100000
        if t == 0:
            nv = max(mg // 8, 32)
            out.append(gnp(nv, 16.0 / (nv - 1), s, name=f"gnp{gi}"))
        elif t == 1:
            sc = int(min(max(round(math.log2(max(mg, 16) / 16.0)), 12), 18))
            gr = rmat(sc, mg, seed=s)
            gr.name = f"rmat{gi}"
            out.append(gr)
        else:
            nv = max(mg // 10, 32)
            gr = rgg(nv, 2, 20.0, s)
            gr.name = f"rgg{gi}"
            out.append(gr)
    return out


def colors(n: int, c: int, seed: int) -> np.ndarray:
    """int32[n]: a colour per vertex, independent and uniform over 0..c-1 (the random
    choice of colorful sparsification, drawn here and passed to both sides)."""
    return rng(seed).integers(0, c, size=n).astype(np.int32)


def relabel(gr: Graph, perm: np.ndarray) -> Graph:
    """Graph with vertex v renamed perm[v]."""
    u, v = gr.edges()
    perm = np.asarray(perm, dtype=np.int64)
    return csr_from_pairs(gr.n, perm[u], perm[v], gr.name + "+relabel")


# ---------------------------------------------------------------- small exact families

def complete(n: int) -> Graph:
    ia, ib = np.triu_indices(n, 1)
    return csr_from_pairs(n, ia, ib, f"K{n}")


def turan(n: int, r: int) -> Graph:
    """Complete r-partite graph with parts as equal as possible (vertex i in part i mod r)."""
    part = np.arange(n) % r
    ia, ib = np.triu_indices(n, 1)
    keep = part[ia] != part[ib]
    return csr_from_pairs(n, ia[keep], ib[keep], f"T({n},{r})")


def cycle(n: int) -> Graph:
    a = np.arange(n)
    return csr_from_pairs(n, a, (a + 1) % n, f"C{n}")


def star(n: int) -> Graph:
    return csr_from_pairs(n, np.zeros(n - 1, np.int64), np.arange(1, n), f"S{n}")


def empty(n: int) -> Graph:
    return csr_from_pairs(n, np.empty(0, np.int64), np.empty(0, np.int64), f"E{n}")


# ---------------------------------------------------------------- named workloads

def config_graph(name: str) -> Graph:
    """The named benchmark workloads at full size.

    c1: G(n=2000, m=20000) + planted K30, seed 1
    c2: R-MAT scale 20, 2^24 samples, seed 2
    c3: Chung-Lu n=2^22, beta=2.1, 2^26 pairs, w_max=4000, 1000 communities of 40-80 at p=0.5, seed 3
    """
    if name == "c1":
        return er_planted(2000, 20000, 30, seed=1)
    if name == "c2":
        return rmat(20, 1 << 24, seed=2)
    if name == "c3":
        return chung_lu(1 << 22, 2.1, 1 << 26, 4000.0, ncomm=1000, seed=3)
    raise KeyError(name)
