"""Thin ctypes binding of libarb.so (include/arb.h).

Argument marshalling only: every step of the path runs in the library's HIP kernels.
PyTorch provides device memory (tensors) and the stream.  Importing this module loads
libarb.so and raises if it is missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libarb.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "arb.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2002_10047_amd.build.build() "
                      "(hipcc --offload-arch=gfx950); there is no CPU fallback")
_lib = ctypes.CDLL(LIB_PATH)

ARB_OK, ARB_EINVAL, ARB_EGRAPH, ARB_EWORKSPACE, ARB_EHIP, ARB_ELIMIT, ARB_EMISMATCH = range(7)
ARB_SCHED_PLAIN, ARB_SCHED_PERSISTENT, ARB_SCHED_LEARNED = range(3)
ARB_ORIENT_PEEL, ARB_ORIENT_DEGREE, ARB_ORIENT_GOODRICH_PSZONA, ARB_ORIENT_KCORE = range(4)


def _define(name):
    m = re.search(r"#define\s+" + name + r"\s+(\d+)", open(HEADER).read()) if os.path.exists(HEADER) else None
    return int(m.group(1)) if m else None


ARB_MAX_K = _define("ARB_MAX_K") or 32
ARB_MAX_LOCAL = _define("ARB_MAX_LOCAL") or 768
ARB_MAX_ROUNDS = _define("ARB_MAX_ROUNDS") or 64
ARB_MLP_PARAMS = _define("ARB_MLP_PARAMS") or 8641
ARB_LEARNED_MIN_DEGREE = _define("ARB_LEARNED_MIN_DEGREE") or 65
ARB_NOALLOC_SCRATCH_BYTES = 64 << 20


class ArbError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {arb_error_string(code)} (code {code})")


class ArbCsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p)]


class ArbOcsr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("indices", ctypes.c_void_p)]


class ArbCountOpts(ctypes.Structure):
    _fields_ = [("schedule", ctypes.c_int), ("split_min_degree", ctypes.c_int),
                ("split_min_cost", ctypes.c_float), ("persist_blocks_per_cu", ctypes.c_int),
                ("chunk_small", ctypes.c_int), ("bitmap_max_span", ctypes.c_int), ("concurrent_tiers", ctypes.c_int),
                ("tier_fill", ctypes.c_int), ("big_max_degree", ctypes.c_int),
                ("mlp_weights", ctypes.c_void_p),
                ("features", ctypes.c_void_p)]


P, I64, I32, SZ, DBL, FLT = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t,
                              ctypes.c_double, ctypes.c_float)
_sigs = {
    "arb_orient_workspace": ([I64, I64], SZ),
    "arb_orient": ([P, DBL, I32, P, P, P, P, P, P, SZ, P], I32),
    "arb_orient_method": ([P, I32, DBL, I32, P, P, P, P, P, P, SZ, P], I32),
    "arb_orient_batch_workspace": ([I64, I64, I64], SZ),
    "arb_orient_batch": ([P, P, I64, I64, DBL, I32, P, P, P, P, P, P, SZ, P], I32),
    "arb_count_batch_workspace": ([I64, I64, I32, I64], SZ),
    "arb_sparsify_workspace": ([I64, I64], SZ),
    "arb_approx_peel_workspace": ([I64, I64, I32], SZ),
    "arb_peel_workspace": ([I64, I64, I32], SZ),
    "arb_peel": ([P, I32, P, P, P, P, SZ, P], I32),
    "arb_approx_peel": ([P, I32, DBL, P, P, P, P, P, SZ, P], I32),
    "arb_sparsify": ([P, P, P, P, P, P, SZ, P], I32),
    "arb_colorful_estimate": ([ctypes.c_uint64, I32, I32], DBL),
    "arb_count_batch_async": ([P, P, I64, I32, P, P, P, P, P, SZ, P], I32),
    "arb_validate": ([P, P, SZ, P], I32),
    "arb_check_oriented": ([P, P, SZ, P], I32),
    "arb_permute_u64": ([P, P, P, I64, P], I32),
    "arb_count_default_opts": ([P], None),
    "arb_count_workspace": ([I64, I64, I32], SZ),
    "arb_count_async": ([P, I32, P, P, P, P, P, P, SZ, P], I32),
    "arb_segment_sum_u64": ([P, P, I64, P, P], I32),
    "arb_count": ([P, I32, P, P, P, SZ, P], ctypes.c_uint64),
    "arb_count_noalloc": ([P, I32, P, P, P, P], I32),
    "arb_count_instrumented": ([P, I32, P, P, P, P, SZ, P], I32),
    "arb_features": ([P, P, P, P, P], I32),
    "arb_features_min_degree": ([P, P, P, I64, P, P], I32),
    "arb_mlp_forward": ([P, P, I64, P, P, P], I32),
    "arb_mlp_workspace": ([I64], SZ),
    "arb_mlp_backward": ([P, P, P, P, I64, P, P, SZ, P], I32),
    "arb_mse_grad": ([P, P, I64, P, P, P], I32),
    "arb_adam_step": ([P, P, P, P, P, FLT, I32, P], I32),
    "arb_to_bf16": ([P, P, I64, P], I32),
    "arb_autotune": ([P, I32, P, I32, P, P, SZ, P], I32),
    "arb_autotune_space": ([I32, I32, P], I32),
    "arb_profile_enable": ([I32], I32),
    "arb_profile_read": ([I32, P, P, P, P, P, P], I32),
    "arb_last_error": ([], I32),
    "arb_error_string": ([I32], ctypes.c_char_p),
}
for _n, (_a, _r) in _sigs.items():
    _f = getattr(_lib, _n)
    _f.argtypes = _a
    _f.restype = _r


def arb_error_string(code: int) -> str:
    return _lib.arb_error_string(int(code)).decode()


def arb_last_error() -> int:
    return int(_lib.arb_last_error())


def _check(rc, where):
    if rc != ARB_OK:
        raise ArbError(rc, where)


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _ws(nbytes: int, device="cuda"):
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def to_device_csr(g, device="cuda"):
    """(offsets int64, indices int32) device tensors of a graphgen.Graph."""
    off = torch.from_numpy(np.ascontiguousarray(g.offsets, np.int64)).to(device)
    idx = torch.from_numpy(np.ascontiguousarray(g.indices, np.int32)).to(device)
    return off, idx


def u64_numpy(t: torch.Tensor) -> np.ndarray:
    """A device int64 tensor holding uint64 bit patterns, as a host uint64 array."""
    return t.cpu().numpy().view(np.uint64)


# ------------------------------------------------------------------ workspace sizes

def arb_orient_workspace(n: int, nnz: int) -> int:
    return int(_lib.arb_orient_workspace(int(n), int(nnz)))


def arb_count_workspace(n: int, m: int, k: int) -> int:
    return int(_lib.arb_count_workspace(int(n), int(m), int(k)))


def arb_mlp_workspace(rows: int) -> int:
    return int(_lib.arb_mlp_workspace(int(rows)))


def arb_count_default_opts():
    o = ArbCountOpts()
    _lib.arb_count_default_opts(ctypes.byref(o))
    return o


# ------------------------------------------------------------------ orientation

def arb_orient(offsets: torch.Tensor, indices: torch.Tensor, eps: float = 1.0, validate: bool = False,
               stream=None):
    """arb_orient: returns dict(ooff, oidx, rank, round, deg_at_peel, stats) device tensors."""
    n = offsets.numel() - 1
    nnz = indices.numel()
    dev = offsets.device
    g = ArbCsr(n, nnz, offsets.data_ptr(), indices.data_ptr() if nnz else 0)
    ooff = torch.empty(n + 1, dtype=torch.int64, device=dev)
    oidx = torch.empty(max(nnz // 2, 1), dtype=torch.int32, device=dev)
    out = ArbOcsr(n, nnz // 2, ooff.data_ptr(), oidx.data_ptr())
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rnd = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    dap = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    stats = torch.empty(2 + ARB_MAX_ROUNDS, dtype=torch.int64, device=dev)
    wsb = _lib.arb_orient_workspace(n, nnz)
    ws = _ws(wsb, dev)
    rc = _lib.arb_orient(ctypes.byref(g), float(eps), int(bool(validate)), ctypes.byref(out), _ptr(rank),
                         _ptr(rnd), _ptr(dap), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "arb_orient")
    return dict(ooff=ooff, oidx=oidx[: nnz // 2], rank=rank[:n], round=rnd[:n], deg_at_peel=dap[:n],
                stats=stats, n=n, m=nnz // 2)


def arb_orient_method(offsets: torch.Tensor, indices: torch.Tensor, method: int, eps: float = 1.0,
                      validate: bool = False, stream=None):
    """arb_orient_method (ARB_ORIENT_*): the same dict as arb_orient."""
    n = offsets.numel() - 1
    nnz = indices.numel()
    dev = offsets.device
    g = ArbCsr(n, nnz, offsets.data_ptr(), indices.data_ptr() if nnz else 0)
    ooff = torch.empty(n + 1, dtype=torch.int64, device=dev)
    oidx = torch.empty(max(nnz // 2, 1), dtype=torch.int32, device=dev)
    out = ArbOcsr(n, nnz // 2, ooff.data_ptr(), oidx.data_ptr())
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rnd = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    dap = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    stats = torch.empty(2 + ARB_MAX_ROUNDS, dtype=torch.int64, device=dev)
    ws = _ws(_lib.arb_orient_workspace(n, nnz), dev)
    rc = _lib.arb_orient_method(ctypes.byref(g), int(method), float(eps), int(bool(validate)), ctypes.byref(out),
                                _ptr(rank), _ptr(rnd), _ptr(dap), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream))
    _check(rc, "arb_orient_method")
    return dict(ooff=ooff, oidx=oidx[: nnz // 2], rank=rank[:n], round=rnd[:n], deg_at_peel=dap[:n],
                stats=stats, n=n, m=nnz // 2)


def arb_orient_batch_workspace(n: int, nnz: int, G: int) -> int:
    return int(_lib.arb_orient_batch_workspace(n, nnz, G))


def arb_orient_batch(offsets: torch.Tensor, indices: torch.Tensor, graph_vtx_offsets, eps: float = 1.0,
                     validate: bool = False, stream=None, max_graph_n=None):
    """arb_orient_batch on a disjoint union; graph_vtx_offsets: int64[G+1], host (numpy)
    or a device tensor (then max_graph_n is required, and nothing is copied, so the call
    can be captured).  Returns the arb_orient dict plus vo (device offsets) and G."""
    n = offsets.numel() - 1
    nnz = indices.numel()
    dev = offsets.device
    if torch.is_tensor(graph_vtx_offsets) and graph_vtx_offsets.is_cuda:
        if max_graph_n is None:
            raise ValueError("max_graph_n is required with device offsets")
        vo = graph_vtx_offsets
        G = vo.numel() - 1
        max_n = int(max_graph_n)
    else:
        vo_h = np.asarray(graph_vtx_offsets, dtype=np.int64)
        G = vo_h.shape[0] - 1
        vo = torch.from_numpy(vo_h.copy()).to(dev)
        max_n = int(np.diff(vo_h).max()) if G > 0 else 0
    g = ArbCsr(n, nnz, offsets.data_ptr(), indices.data_ptr() if nnz else 0)
    ooff = torch.empty(n + 1, dtype=torch.int64, device=dev)
    oidx = torch.empty(max(nnz // 2, 1), dtype=torch.int32, device=dev)
    out = ArbOcsr(n, nnz // 2, ooff.data_ptr(), oidx.data_ptr())
    rank = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    rnd = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    dap = torch.empty(max(n, 1), dtype=torch.int32, device=dev)
    stats = torch.empty(2 + ARB_MAX_ROUNDS, dtype=torch.int64, device=dev)
    ws = _ws(_lib.arb_orient_batch_workspace(n, nnz, max(G, 1)), dev)
    rc = _lib.arb_orient_batch(ctypes.byref(g), _ptr(vo), G, max_n, float(eps), int(bool(validate)),
                               ctypes.byref(out), _ptr(rank), _ptr(rnd), _ptr(dap), _ptr(stats), _ptr(ws),
                               ws.numel(), _stream(stream))
    _check(rc, "arb_orient_batch")
    return dict(ooff=ooff, oidx=oidx[: nnz // 2], rank=rank[:n], round=rnd[:n], deg_at_peel=dap[:n],
                stats=stats, n=n, m=nnz // 2, vo=vo, G=G)


def arb_sparsify_workspace(n: int, nnz: int) -> int:
    return int(_lib.arb_sparsify_workspace(n, nnz))


def arb_sparsify(offsets, indices, colors, stream=None):
    """Colorful sparsification: (offsets, indices) of the graph that keeps the edges whose
    endpoints share a colour (colors: device int32[n])."""
    n = offsets.numel() - 1
    nnz = indices.numel()
    dev = offsets.device
    g = ArbCsr(n, nnz, offsets.data_ptr(), indices.data_ptr() if nnz else 0)
    out_off = torch.empty(n + 1, dtype=torch.int64, device=dev)
    out_idx = torch.empty(max(nnz, 1), dtype=torch.int32, device=dev)
    out_nnz = ctypes.c_int64(0)
    ws = _ws(_lib.arb_sparsify_workspace(n, nnz), dev)
    _check(_lib.arb_sparsify(ctypes.byref(g), _ptr(colors), _ptr(out_off), _ptr(out_idx), ctypes.byref(out_nnz),
                             _ptr(ws), ws.numel(), _stream(stream)), "arb_sparsify")
    return out_off, out_idx[: out_nnz.value]


def arb_approx_peel_workspace(n: int, m: int, k: int) -> int:
    return int(_lib.arb_approx_peel_workspace(n, m, int(k)))


def arb_approx_peel(ooff, oidx, k, eps=1.0, opts=None, stream=None):
    """arb-approx-peel: (best density, rounds, best mask int32[n] in rank space)."""
    dg = _ocsr(ooff, oidx)
    n = dg.n
    mask = torch.empty(max(n, 1), dtype=torch.int32, device=ooff.device)
    ws = _ws(_lib.arb_approx_peel_workspace(n, dg.m, int(k)), ooff.device)
    dens = ctypes.c_double(0.0)
    rounds = ctypes.c_int64(0)
    _check(_lib.arb_approx_peel(ctypes.byref(dg), int(k), float(eps), ctypes.byref(opts) if opts is not None else None,
                                ctypes.byref(dens), ctypes.byref(rounds), _ptr(mask), _ptr(ws), ws.numel(),
                                _stream(stream)), "arb_approx_peel")
    return dens.value, rounds.value, mask[:n]


def arb_peel_workspace(n: int, m: int, k: int) -> int:
    return int(_lib.arb_peel_workspace(n, m, int(k)))


def arb_peel(ooff, oidx, k, stream=None):
    """arb-peel: (best density, rounds, round of each vertex int32[n] in rank space)."""
    dg = _ocsr(ooff, oidx)
    n = dg.n
    rnd = torch.empty(max(n, 1), dtype=torch.int32, device=ooff.device)
    ws = _ws(_lib.arb_peel_workspace(n, dg.m, int(k)), ooff.device)
    dens = ctypes.c_double(0.0)
    rounds = ctypes.c_int64(0)
    _check(_lib.arb_peel(ctypes.byref(dg), int(k), ctypes.byref(dens), ctypes.byref(rounds), _ptr(rnd), _ptr(ws),
                         ws.numel(), _stream(stream)), "arb_peel")
    return dens.value, rounds.value, rnd[:n]


def arb_colorful_estimate(count: int, colors: int, k: int) -> float:
    y = float(_lib.arb_colorful_estimate(int(count), int(colors), int(k)))
    _check(arb_last_error(), "arb_colorful_estimate")
    return y


def arb_validate(offsets, indices, stream=None) -> int:
    n = offsets.numel() - 1
    g = ArbCsr(n, indices.numel(), offsets.data_ptr(), indices.data_ptr() if indices.numel() else 0)
    ws = _ws(4096, offsets.device)
    return int(_lib.arb_validate(ctypes.byref(g), _ptr(ws), ws.numel(), _stream(stream)))


def _ocsr(ooff, oidx):
    n = ooff.numel() - 1
    m = oidx.numel()
    return ArbOcsr(n, m, ooff.data_ptr(), oidx.data_ptr() if m else 0)


def arb_check_oriented(ooff, oidx, stream=None) -> int:
    dg = _ocsr(ooff, oidx)
    ws = _ws(4096, ooff.device)
    return int(_lib.arb_check_oriented(ctypes.byref(dg), _ptr(ws), ws.numel(), _stream(stream)))


def arb_permute_u64(rank, values, stream=None):
    out = torch.empty_like(values)
    _check(_lib.arb_permute_u64(_ptr(rank), _ptr(values), _ptr(out), rank.numel(), _stream(stream)),
           "arb_permute_u64")
    return out


# ------------------------------------------------------------------ counting

def count_opts(schedule=ARB_SCHED_PERSISTENT, split_min_degree=0, split_min_cost=0.0,
               persist_blocks_per_cu=8, chunk_small=16, mlp_weights=None, features=None, bitmap_max_span=1 << 30,
               concurrent_tiers=1, tier_fill=100, big_max_degree=-1):
    o = ArbCountOpts()
    _lib.arb_count_default_opts(ctypes.byref(o))
    o.schedule = int(schedule)
    o.split_min_degree = int(split_min_degree)
    o.split_min_cost = float(split_min_cost)
    o.persist_blocks_per_cu = int(persist_blocks_per_cu)
    o.chunk_small = int(chunk_small)
    o.bitmap_max_span = int(bitmap_max_span)
    o.concurrent_tiers = int(concurrent_tiers)
    o.tier_fill = int(tier_fill)
    o.big_max_degree = int(big_max_degree)
    o.mlp_weights = mlp_weights.data_ptr() if mlp_weights is not None else None
    o.features = features.data_ptr() if features is not None else None
    o._keep = (mlp_weights, features)
    return o


def opts_dict(o):
    return {"schedule": o.schedule, "split_min_degree": o.split_min_degree, "split_min_cost": o.split_min_cost,
            "persist_blocks_per_cu": o.persist_blocks_per_cu, "chunk_small": o.chunk_small,
            "bitmap_max_span": o.bitmap_max_span, "concurrent_tiers": o.concurrent_tiers, "tier_fill": o.tier_fill,
            "big_max_degree": o.big_max_degree}


def arb_autotune(ooff, oidx, k, opts, trials=3, ws=None, stream=None):
    """Tunes opts in place (see include/arb.h); returns the best time in ms."""
    dg = _ocsr(ooff, oidx)
    if ws is None:
        ws = CountWorkspace(ooff, oidx, k)
    ms = ctypes.c_float(0.0)
    _check(_lib.arb_autotune(ctypes.byref(dg), int(k), ctypes.byref(opts), int(trials), ctypes.byref(ms), _ptr(ws.buf),
                             ws.buf.numel(), _stream(stream)), "arb_autotune")
    return float(ms.value)


TUNE_DIMS = {"split_min_degree": 0, "split_min_cost": 1, "persist_blocks_per_cu": 2, "chunk_small": 3,
             "bitmap_max_span": 4, "concurrent_tiers": 5, "tier_fill": 6, "big_max_degree": 7}


def arb_autotune_space():
    """{option name: candidate values} of arb_autotune's search."""
    out = {}
    for name, dim in TUNE_DIMS.items():
        cnt = _lib.arb_autotune_space(dim, 0, None)
        if cnt < 0:
            raise ArbError(arb_last_error(), "arb_autotune_space")
        buf = (ctypes.c_double * max(cnt, 1))()
        _lib.arb_autotune_space(dim, cnt, buf)
        out[name] = [float(x) if name == "split_min_cost" else int(x) for x in buf[:cnt]]
    return out


class CountWorkspace:
    """Reusable device workspace for arb_count_async on one graph."""

    def __init__(self, ooff, oidx, k):
        n = ooff.numel() - 1
        self.bytes = int(_lib.arb_count_workspace(n, oidx.numel(), int(k)))
        self.buf = _ws(self.bytes, ooff.device)


def arb_count_async(ooff, oidx, k, total=None, per_vertex=None, work=None, opts=None, ws=None, stream=None,
                    per_root=None):
    """Enqueue arb_count_async; returns the device total tensor (int64 holding uint64)."""
    dg = _ocsr(ooff, oidx)
    if ws is None:
        ws = CountWorkspace(ooff, oidx, k)
    if total is None:
        total = torch.empty(1, dtype=torch.int64, device=ooff.device)
    rc = _lib.arb_count_async(ctypes.byref(dg), int(k), _ptr(total), _ptr(per_vertex), _ptr(per_root), _ptr(work),
                              ctypes.byref(opts) if opts is not None else None, _ptr(ws.buf), ws.buf.numel(),
                              _stream(stream))
    _check(rc, "arb_count_async")
    return total


def arb_count_instrumented(ooff, oidx, k, cycles=False, opts=None, ws=None, stream=None):
    """(work, cycles or None): per-root work measure and, if asked, clock cycles per root
    (device int64 tensors holding uint64)."""
    dg = _ocsr(ooff, oidx)
    n = ooff.numel() - 1
    if ws is None:
        ws = CountWorkspace(ooff, oidx, k)
    work = torch.empty(max(n, 1), dtype=torch.int64, device=ooff.device)
    cyc = torch.empty(max(n, 1), dtype=torch.int64, device=ooff.device) if cycles else None
    _check(_lib.arb_count_instrumented(ctypes.byref(dg), int(k), _ptr(work), _ptr(cyc),
                                       ctypes.byref(opts) if opts is not None else None, _ptr(ws.buf), ws.buf.numel(),
                                       _stream(stream)), "arb_count_instrumented")
    return work[:n], (cyc[:n] if cyc is not None else None)


def arb_count_noalloc(ooff, oidx, k, total=None, per_vertex=None, opts=None, stream=None):
    """Enqueue arb_count_noalloc (no workspace argument); returns the device total tensor."""
    dg = _ocsr(ooff, oidx)
    if total is None:
        total = torch.empty(1, dtype=torch.int64, device=ooff.device)
    rc = _lib.arb_count_noalloc(ctypes.byref(dg), int(k), _ptr(total), _ptr(per_vertex),
                                ctypes.byref(opts) if opts is not None else None, _stream(stream))
    _check(rc, "arb_count_noalloc")
    return total


def arb_count_batch_workspace(n: int, m: int, k: int, G: int) -> int:
    return int(_lib.arb_count_batch_workspace(n, m, k, G))


def arb_count_batch_async(ooff, oidx, vo, k, totals=None, total=None, per_vertex=None, opts=None, ws=None,
                          stream=None):
    """Per-graph totals (device int64[G] holding uint64) of a batch from arb_orient_batch;
    vo: its device vertex offsets; ws: a byte tensor of arb_count_batch_workspace bytes."""
    dg = _ocsr(ooff, oidx)
    G = vo.numel() - 1
    if ws is None:
        ws = _ws(_lib.arb_count_batch_workspace(dg.n, dg.m, int(k), G), ooff.device)
    if totals is None:
        totals = torch.empty(max(G, 1), dtype=torch.int64, device=ooff.device)
    rc = _lib.arb_count_batch_async(ctypes.byref(dg), _ptr(vo), G, int(k), _ptr(per_vertex), _ptr(totals),
                                    _ptr(total), ctypes.byref(opts) if opts is not None else None, _ptr(ws),
                                    ws.numel(), _stream(stream))
    _check(rc, "arb_count_batch_async")
    return totals[:G]


def arb_count(ooff, oidx, k, per_vertex: bool = False, opts=None, ws=None, stream=None):
    """Synchronous arb_count: returns the total (int), or (total, per_vertex uint64 numpy)."""
    dg = _ocsr(ooff, oidx)
    n = ooff.numel() - 1
    if ws is None:
        ws = CountWorkspace(ooff, oidx, k)
    pv = torch.empty(max(n, 1), dtype=torch.int64, device=ooff.device) if per_vertex else None
    t = _lib.arb_count(ctypes.byref(dg), int(k), _ptr(pv), ctypes.byref(opts) if opts is not None else None,
                       _ptr(ws.buf), ws.buf.numel(), _stream(stream))
    err = arb_last_error()
    _check(err, "arb_count")
    if per_vertex:
        return int(t), u64_numpy(pv)[:n]
    return int(t)


def arb_profile_enable(on: bool = True):
    _check(_lib.arb_profile_enable(int(bool(on))), "arb_profile_enable")


def arb_profile_read(max_entries: int = 256):
    """List of dicts (tier, k, per_vertex, instrumented, launches, total_ms) accumulated
    since arb_profile_enable(True)."""
    T = (ctypes.c_int32 * max_entries)
    tier, k, pv, ins = T(), T(), T(), T()
    la = (ctypes.c_int64 * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    nent = _lib.arb_profile_read(max_entries, tier, k, pv, ins, la, ms)
    if nent < 0:
        raise ArbError(arb_last_error(), "arb_profile_read")
    return [dict(tier=tier[i], k=k[i], per_vertex=pv[i], instrumented=ins[i], launches=la[i], total_ms=ms[i])
            for i in range(min(nent, max_entries))]


def arb_segment_sum_u64(values, offsets, stream=None):
    """Per-segment sums of a device uint64 (int64-typed) tensor; offsets: device int64[G+1]."""
    G = offsets.numel() - 1
    out = torch.empty(max(G, 1), dtype=torch.int64, device=values.device)
    _check(_lib.arb_segment_sum_u64(_ptr(values), _ptr(offsets), G, _ptr(out), _stream(stream)),
           "arb_segment_sum_u64")
    return out[:G]


# ------------------------------------------------------------------ learned schedule

def _features_out(ooff, out):
    n = ooff.numel() - 1
    if out is None:
        return torch.empty(max(n, 1) * 3, dtype=torch.float32, device=ooff.device)
    if out.dtype != torch.float32 or not out.is_contiguous() or out.numel() < max(n, 1) * 3:
        raise ValueError("out must be a contiguous float32 tensor of at least 3n elements")
    return out


def arb_features(ooff, oidx, round_orig=None, rank=None, stream=None, out=None):
    """Per-root features [n, 3]; out: optional float32 device tensor of at least 3n elements."""
    n = ooff.numel() - 1
    feat = _features_out(ooff, out)
    dg = _ocsr(ooff, oidx)
    _check(_lib.arb_features(ctypes.byref(dg), _ptr(round_orig), _ptr(rank), _ptr(feat), _stream(stream)),
           "arb_features")
    return feat.view(-1)[: 3 * n].view(n, 3)


def arb_features_min_degree(ooff, oidx, round_orig, rank, min_degree, stream=None, out=None):
    """The rows of arb_features for roots with at least min_degree out-neighbours; the other
    rows keep what `out` held (uninitialised without `out`)."""
    n = ooff.numel() - 1
    feat = _features_out(ooff, out)
    dg = _ocsr(ooff, oidx)
    _check(_lib.arb_features_min_degree(ctypes.byref(dg), _ptr(round_orig), _ptr(rank), int(min_degree),
                                        _ptr(feat), _stream(stream)), "arb_features_min_degree")
    return feat.view(-1)[: 3 * n].view(n, 3)


def arb_mlp_forward(w_bf16, x, want_act=False, stream=None):
    rows = x.shape[0]
    y = torch.empty(max(rows, 1), dtype=torch.float32, device=x.device)
    act = torch.empty(max(rows, 1) * 192, dtype=torch.float32, device=x.device) if want_act else None
    _check(_lib.arb_mlp_forward(_ptr(w_bf16), _ptr(x), rows, _ptr(y), _ptr(act), _stream(stream)),
           "arb_mlp_forward")
    return (y[:rows], act) if want_act else y[:rows]


def arb_mlp_backward(w_bf16, x, act, dy, stream=None):
    rows = x.shape[0]
    grad = torch.empty(ARB_MLP_PARAMS, dtype=torch.float32, device=x.device)
    ws = _ws(_lib.arb_mlp_workspace(rows), x.device)
    _check(_lib.arb_mlp_backward(_ptr(w_bf16), _ptr(x), _ptr(act), _ptr(dy), rows, _ptr(grad), _ptr(ws),
                                 ws.numel(), _stream(stream)), "arb_mlp_backward")
    return grad


def arb_mse_grad(y, target, stream=None):
    rows = y.numel()
    dy = torch.empty_like(y)
    loss = torch.empty(1, dtype=torch.float32, device=y.device)
    _check(_lib.arb_mse_grad(_ptr(y), _ptr(target), rows, _ptr(dy), _ptr(loss), _stream(stream)), "arb_mse_grad")
    return dy, loss


def arb_adam_step(w, w_bf16, grad, m, v, lr, step, stream=None):
    _check(_lib.arb_adam_step(_ptr(w), _ptr(w_bf16), _ptr(grad), _ptr(m), _ptr(v), float(lr), int(step),
                              _stream(stream)), "arb_adam_step")


def arb_to_bf16(w, stream=None):
    out = torch.empty(w.numel(), dtype=torch.int16, device=w.device)
    _check(_lib.arb_to_bf16(_ptr(w), _ptr(out), w.numel(), _stream(stream)), "arb_to_bf16")
    return out


def exported_symbols():
    """Function names declared in include/arb.h."""
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(arb_[a-z0-9_]+)\s*\(", src)))
