#!/usr/bin/env python3
"""Throughput benchmark of the arb-count hot path on one MI355X.

Headline workload (the largest single-GPU configuration): the 3-D random geometric graph
on the unit torus, 2^24 vertices, mean degree 40 (~335M edges, counter-based stream, seed
52, built on the GPU), k = 5, 6, 7 with per-vertex counts.  One step = the whole hot path
on the resident graph: arb_orient (eps = 1), the scheduling features, and arb_count for
k = 5, 6 and 7 with per-vertex counts (exact totals).  `value` = k-cliques counted per
second of step time (sum over the three k).

Also reported: R-MAT scale 26 (2^30 samples, seed 51, ~1.05 billion edges) at k = 4 and
R-MAT scale 20 (2^24 samples, seed 2) at k = 3, 4, 5 -- orientation and count times per
schedule (learned, degree, plain), each count checked equal across schedules -- the
roofline of the headline's dominant counting kernel, the CPU-oracle baseline and the
studies of the paper's other rows (sparsification, orderings, approximate peeling).

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0                 # MI355X HBM3E
# plain 32-bit integer VALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# LDS: 128 B/clk/CU (the CDNA3 figure) x 256 CUs x 2.4 GHz; the probe's measurement is
# used when larger
SPEC_LDS_GBS = 128 * 256 * 2.4e9 / 1e9
TIER_W = [2, 4, 8, 12, 16, 24]
TIER_CAP = [64, 128, 256, 384, 512, 768]
CPU_THREADS = 16                      # the host-core share of one GPU on the benchmark boxes


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--eps", type=float, default=1.0)
    ap.add_argument("--schedule", default="learned", choices=["plain", "degree", "learned"])
    ap.add_argument("--no-tune", action="store_true", help="library default options, no autotuning")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if options are cached")
    ap.add_argument("--tune-cache", default="", help="tuned-options cache file (default: the package's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the headline's timed steps (profiling runs): no other schedule, workload or study")
    ap.add_argument("--no-studies", action="store_true", help="skip the studies of the other rows")
    ap.add_argument("--no-rmat26", action="store_true", help="skip the R-MAT scale-26 workload")
    ap.add_argument("--only", default="", choices=["", "rmat26", "rmat20"],
                    help="profiling runs: only this workload's timed steps with the chosen schedule (no JSON line)")
    ap.add_argument("--cpu-seconds", type=float, default=30.0, help="expected CPU-baseline time (sets its limit)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (counter calibration)")
    return ap.parse_args()


# ---------------------------------------------------------------------- helpers

def golden(name):
    p = os.path.join(ROOT, "tests", "golden", "fullsize_totals.json")
    try:
        with open(p) as f:
            return json.load(f).get(name)
    except OSError:
        return None


def tier_of_fill(d, fill):
    """numpy counterpart of the scheduler's tier rule: the first tier whose capacity times
    fill/100 holds d (the largest if none), 6 above the LDS tiers."""
    import numpy as np
    cap = np.array(TIER_CAP)
    t0 = np.searchsorted(cap, d, side="left")       # smallest tier that fits
    t = np.full(d.shape, len(cap) - 1)
    for i in range(len(cap) - 1, -1, -1):
        t = np.where((i >= t0) & (d * 100 <= cap[i] * fill), i, t)
    return np.where(t0 >= len(cap), len(cap), t)


def algorithmic_units(arb, o, ks, np):
    """Per-root algorithmic units from the instrumented count: gather words and the
    numbers of search-tree nodes (c_j(v), j-cliques inside G[N+(v)], summed over j <= k-2)."""
    import torch
    ooff_t = o["ooff"]
    dt = ooff_t[1:] - ooff_t[:-1]
    # gather words of root v: sum of d+(u) over u in N+(v), as a segmented sum on the GPU
    cs = torch.zeros(o["oidx"].numel() + 1, dtype=torch.int64, device=ooff_t.device)
    torch.cumsum(dt[o["oidx"].long()], 0, out=cs[1:])
    gather = (cs[ooff_t[1:]] - cs[ooff_t[:-1]]).cpu().numpy()
    del cs
    d = dt.cpu().numpy()
    n = len(d)
    W = (d + 31) // 32
    nodes = {}
    for k in sorted(set(ks) | {k - 1 for k in ks if k >= 4} | {3}):
        work = torch.empty(n, dtype=torch.int64, device="cuda")
        arb.arb_count_async(o["ooff"], o["oidx"], k, work=work)
        torch.cuda.synchronize()
        wk = work.cpu().numpy()
        del work
        live = d >= k - 1
        nd = np.zeros(n, np.int64)
        nd[live] = (wk[live] - gather[live]) // W[live]
        nodes[k] = nd
    return d, W, gather, nodes


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_child(path, ks, threads):
    """Child process: the CPU oracle (Chiba-Nishizeki, OpenMP over roots) on the whole
    sample graph for each k on `threads` host threads, then k = 3 on one thread (the
    oracle's authority build).  Prints one JSON line per run."""
    import numpy as np
    import oracle
    from paper_2002_10047_amd import graphgen as gg
    z = np.load(path)
    g = gg.Graph(int(z["n"]), z["offsets"], z["indices"])
    for k, th in [(k, threads) for k in ks] + [(3, 1)]:
        t1 = time.time()
        c = oracle.count(g, k, nthreads=th)
        print(json.dumps({"k": k, "threads": th, "count": c, "seconds": time.time() - t1}), flush=True)


def cpu_baseline(ks, seconds, exact, n_full):
    """The CPU oracle on a bounded sample of the headline workload: the whole 3-D torus RGG
    of the same recipe (mean degree 40, the counter-based stream, seed 52) with 2^19
    vertices, 1/32 of the headline's.  Its cliques per vertex match the full graph's (the
    recipe is scale-free at fixed mean degree; the counts times 32 are compared with the
    oracle's full-graph totals), so cliques/s on it stand for the oracle's rate on the
    full graph.  CPU_THREADS threads (the host-core share of one GPU), plus k = 3 on one
    thread."""
    import subprocess
    import tempfile
    import numpy as np
    from paper_2002_10047_amd import graphgen as gg
    ns = 1 << 20
    n, off, idx = gg.rgg_cb_device(ns, 40.0, seed=52)
    off_h, idx_h = off.cpu().numpy(), idx.cpu().numpy()
    del off, idx
    out = {"unit": "k-cliques/s", "cores": CPU_THREADS, "kind": "oracle", "nproc": os.cpu_count(),
           "cpu_model": cpu_model(), "per_k": {}}
    lines = []
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "g.npz")
        np.savez(path, n=ns, offsets=off_h, indices=idx_h)
        try:
            r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", path,
                                ",".join(str(k) for k in ks), str(CPU_THREADS)], capture_output=True, text=True,
                               timeout=max(60.0, 6 * seconds))
            lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
        except subprocess.TimeoutExpired as e:
            lines = [l for l in (e.stdout or b"").decode().splitlines() if l.startswith("{")]
    cnt = tsum = 0.0
    for l in lines:
        e = json.loads(l)
        if e["threads"] == 1:
            out["single_thread_k3"] = {"count": e["count"], "seconds": e["seconds"],
                                       "cliques_per_s": e["count"] / e["seconds"]}
            continue
        k = e["k"]
        pk = {"count": e["count"], "seconds": e["seconds"], "cliques_per_s": e["count"] / e["seconds"]}
        if exact and str(k) in exact:
            pk["count_x_scale_over_exact"] = e["count"] * (n_full / ns) / exact[str(k)]
        out["per_k"][str(k)] = pk
        cnt += e["count"]
        tsum += e["seconds"]
        log(f"cpu oracle k={k}: {pk}")
    if tsum <= 0:
        return None
    out["value"] = cnt / tsum
    out["sample"] = (f"the whole 3-D torus RGG of the headline's recipe with 2^20 vertices (mean degree 40, seed 52; "
                     f"1/{n_full // ns} of the headline graph), k = {ks}, Chiba-Nishizeki oracle on {CPU_THREADS} "
                     "threads; value = sum of counts / sum of seconds; count_x_scale_over_exact compares its counts "
                     "times the size ratio with the oracle's totals of the full graph")
    return out


def copy_calibration(a, torch):
    """One plain device copy of a known size, for scaling the HBM byte counters."""
    if not a.copy_calibration_mib:
        return
    nb = a.copy_calibration_mib << 20
    # the copied range is written first and then evicted from the 256 MB Infinity Cache
    # by writing 1 GiB behind it, so that the copy's reads come from HBM
    big = torch.ones(nb // 4 + (1 << 28), dtype=torch.float32, device="cuda")
    src = big[: nb // 4]
    dst = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy calibration: {nb} bytes read and {nb} bytes written once")


def measure_peaks(torch):
    """LDS read and device copy bandwidth from the project's probes (libarb_probe.so)."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2002_10047_amd", "libarb_probe.so"))
    lib.arb_probe_lds_read.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                       ctypes.c_void_p]
    lib.arb_probe_copy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p,
                                   ctypes.c_void_p]
    props = torch.cuda.get_device_properties(0)
    cus = props.multi_processor_count
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    scratch = torch.empty(cus * 2 * 1024, dtype=torch.int32, device="cuda")
    lds = []
    for bpc in (1, 2):
        v = ctypes.c_double(0.0)
        if lib.arb_probe_lds_read(ctypes.c_void_p(scratch.data_ptr()), scratch.numel(), bpc, ctypes.byref(v),
                                  stream) == 0:
            lds.append(v.value / 1e9)
    nb = 1 << 30
    src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    v = ctypes.c_double(0.0)
    cp = v.value / 1e9 if lib.arb_probe_copy(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), nb, 5,
                                             ctypes.byref(v), stream) == 0 else None
    del src, dst
    return {"lds_read_GBs": max(lds) if lds else None, "copy_GBs": cp if cp else None, "cus": cus}


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("count_kernels.h", "count.hip", "count_big.hip"):
        with open(os.path.join(ROOT, "paper_2002_10047_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_counters(kernel, workload):
    """The committed rocprofv3 counter summary of `kernel` on `workload` (HBM bytes per
    launch, VALU and LDS instruction counts), if it was taken on the current kernel
    sources; else None."""
    p = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    w = t.get("workloads", {}).get(workload)
    if w is None or w.get("source_hash") != kernel_source_hash():
        return None
    return w.get("kernels", {}).get(kernel)


def measured_traffic(kernel, workload):
    e = measured_counters(kernel, workload)
    return None if e is None else e.get("hbm_bytes_per_launch")


def kernel_symbol(tier, k, pv):
    if tier > len(TIER_W):
        return f"k_count_big<{int(pv)},0> (overflowed pair items)"
    if tier == len(TIER_W):
        return f"k_count_big<{int(pv)},0>"
    return f"k_count<{TIER_W[tier]},{max(1, min(k - 3, 8))},{int(pv)},0>"


def roofline(arb, np, torch, o, ks, pv, opts_of_k, prof, workload):
    """Per counting kernel of the timed steps: launches, time, algorithmic HBM bytes, VALU
    ops and LDS bytes (per-root formulas summed over the roots the kernel processed).  The
    dominant kernel is the one with the largest total time over the timed steps."""
    d, W, gather, nodes = algorithmic_units(arb, o, ks, np)
    per_sym = {}
    phase = {}
    for e in prof:
        k, ti = e["k"], e["tier"]
        op = opts_of_k[k]
        live = d >= k - 1
        td = tier_of_fill(d, op.tier_fill)
        sel = live & (td == ti)
        hbm = float(4 * (d[sel] + 4 * d[sel] + gather[sel]).sum() + 16 * sel.sum())
        if pv:
            hbm += float(8 * (d[sel] + 1).sum())           # one u64 update per member and root
        alu = lds = 0.0
        if k >= 4:
            ck2 = nodes[k][sel] - nodes[k - 1][sel]          # c_{k-2}(v)
            deep = nodes[k][sel] - d[sel]                    # sum_{j=2}^{k-2} c_j(v)
            # every node of depth >= 2 ANDs W words; nodes of depth k-2 also popcount them
            alu = float((W[sel] * (deep + ck2)).sum())
            # rows built (d), a row read and a set written per internal node (depth 1..k-3),
            # a row read per node of depth k-2
            lds = float((4 * W[sel] * (d[sel] + nodes[k - 1][sel] + nodes[k][sel])).sum())
        sym = kernel_symbol(ti, k, pv)
        s_ = per_sym.setdefault(sym, dict(launches=0, ms=0.0, hbm=0.0, alu=0.0, lds=0.0, parts=[]))
        s_["launches"] += e["launches"]
        s_["ms"] += e["total_ms"]
        s_["hbm"] += e["launches"] * hbm
        s_["alu"] += e["launches"] * alu
        s_["lds"] += e["launches"] * lds
        ph = phase.setdefault(k, dict(alu=0.0, lds=0.0, hbm=0.0))
        ph["alu"] += alu
        ph["lds"] += lds
        ph["hbm"] += hbm
        s_["parts"].append(f"k={k}: {e['launches']} launches, {e['total_ms'] / e['launches']:.3f} ms avg")
    peaks = measure_peaks(torch)
    peak_lds = max(SPEC_LDS_GBS, peaks["lds_read_GBs"] or 0.0)
    log(f"probes: LDS read {peaks['lds_read_GBs']:.0f} GB/s, device copy {peaks['copy_GBs']:.0f} GB/s "
        f"(LDS peak used {peak_lds:.0f} GB/s)")
    kernels = {}
    best = None
    for sym, v in sorted(per_sym.items()):
        sec = v["ms"] / 1e3
        fr = {"hbm": v["hbm"] / sec / 1e9 / PEAK_HBM_GBS, "alu": v["alu"] / sec / 1e12 / PEAK_ALU_TOPS,
              "lds": v["lds"] / sec / 1e9 / peak_lds}
        kernels[sym] = {"launches": v["launches"], "avg_ms": v["ms"] / v["launches"], "total_ms": v["ms"],
                        "fracs": fr}
        log(f"  {sym}: {v['launches']} launches, avg {v['ms'] / v['launches']:.3f} ms ({'; '.join(v['parts'])}), "
            f"HBM {fr['hbm']:.2%}, ALU {fr['alu']:.2%}, LDS {fr['lds']:.2%}")
        # a launch that processed no item (the global-scratch kernel on a graph without
        # large roots) only waited for CUs beside the tiers: never the dominant kernel
        if v["hbm"] + v["alu"] + v["lds"] > 0 and (best is None or v["ms"] > best[1]["ms"]):
            best = (sym, v, fr)
    out = None
    if best:
        sym, v, fr = best
        bound = max(fr, key=fr.get)
        per = {"hbm": v["hbm"], "alu": v["alu"], "lds": v["lds"]}[bound] / v["launches"]
        sec = v["ms"] / 1e3 / v["launches"]
        unit, scale, peak = {"hbm": ("GB/s", 1e9, PEAK_HBM_GBS), "alu": ("Tops/s", 1e12, PEAK_ALU_TOPS),
                             "lds": ("GB/s", 1e9, peak_lds)}[bound]
        mc = measured_counters(sym, workload)
        out = {"bound": bound, "achieved": per / sec / scale, "peak": peak, "unit": unit, "frac": fr[bound],
               "traffic": measured_traffic(sym, workload), "kernel": sym, "launches": v["launches"],
               "measured": None if mc is None else {k: mc.get(k) for k in ("valu_issue_frac", "valu_insts",
                                                                           "lds_insts", "avg_ms")},
               "launch_ms": v["ms"] / v["launches"], "algorithmic_per_launch": per, "fracs": fr,
               "rule": "the counting kernel with the largest total time over the timed steps (kernels that "
                       "processed no item excluded)",
               "peaks_measured": peaks, "kernels": kernels}
    return out, phase


# ---------------------------------------------------------------------- workloads

class Workload:
    """A resident graph, its orientation, workspaces and per-schedule options for ks."""

    def __init__(self, arb, torch, name, n, off, idx, ks, eps, pv, a, log_prefix, tune=True):
        from paper_2002_10047_amd import learn, tuning
        self.arb, self.torch, self.name, self.n, self.off, self.idx, self.ks, self.eps, self.pv = \
            arb, torch, name, n, off, idx, ks, eps, pv
        self.o = arb.arb_orient(off, idx, eps=eps)
        self.m = idx.numel() // 2
        self.wss = {k: arb.CountWorkspace(self.o["ooff"], self.o["oidx"], k) for k in ks}
        self.totals = {k: torch.empty(1, dtype=torch.int64, device="cuda") for k in ks}
        self.pvs = {k: torch.empty(n, dtype=torch.int64, device="cuda") for k in ks} if pv else {}
        self.weights = {k: learn.load_weights(k) for k in ks}
        missing = [k for k in ks if self.weights[k] is None]
        if missing:
            raise SystemExit(f"no trained cost model for k={missing}: run python -m paper_2002_10047_amd.train_cost")
        self.feat = arb.arb_features(self.o["ooff"], self.o["oidx"], self.o["round"], self.o["rank"])
        t_tune = time.time()
        cache = a.tune_cache or tuning.CACHE
        self.opts = {}
        for sname in ("degree", "learned"):
            per_k = {}
            for k in ks:
                w = self.weights[k] if sname == "learned" else None
                f = self.feat if sname == "learned" else None
                if a.no_tune or not tune:
                    op = arb.count_opts(schedule=tuning.SCHEDULES[sname], mlp_weights=w, features=f)
                else:
                    op, _ = tuning.tuned_opts(self.o["ooff"], self.o["oidx"], k, sname, mlp_weights=w, features=f,
                                              ws=self.wss[k], retune=a.retune, path=cache, log=log)
                per_k[k] = op
            self.opts[sname] = per_k
        self.opts["plain"] = {k: arb.count_opts(schedule=arb.ARB_SCHED_PLAIN) for k in ks}
        log(f"{log_prefix}: options ready in {time.time() - t_tune:.1f}s")

    def step(self, sname, orient=True):
        arb = self.arb
        oo = arb.arb_orient(self.off, self.idx, eps=self.eps) if orient else self.o
        if sname == "learned":
            # the schedule reads the cost of roots above the 64-tier only
            f = (arb.arb_features_min_degree(oo["ooff"], oo["oidx"], oo["round"], oo["rank"],
                                             arb.ARB_LEARNED_MIN_DEGREE) if orient else self.feat)
            for k in self.ks:
                self.opts[sname][k].features = f.data_ptr()
                self.opts[sname][k]._keep = (self.weights[k], f)
        for k in self.ks:
            arb.arb_count_async(oo["ooff"], oo["oidx"], k, total=self.totals[k], per_vertex=self.pvs.get(k),
                                opts=self.opts[sname][k], ws=self.wss[k])
        return oo

    def read_totals(self):
        import numpy as np
        return {k: int(self.totals[k].cpu().numpy().view(np.uint64)[0]) for k in self.ks}

    def timed(self, sname, steps, warmup, orient=True):
        torch = self.torch
        for _ in range(warmup):
            self.step(sname, orient)
            torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(steps):
            self.step(sname, orient)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / steps
        tot = self.read_totals()
        log(f"{self.name} {sname}: {ms:.3f} ms/step over {steps} steps, totals {tot}")
        return ms, tot

    def phases(self, sname):
        """orientation and per-k count times of one step (HIP events on the stream)."""
        torch = self.torch
        ks = self.ks
        e = [torch.cuda.Event(enable_timing=True) for _ in range(2 + 2 * len(ks))]
        torch.cuda.synchronize()
        e[0].record()
        o = self.arb.arb_orient(self.off, self.idx, eps=self.eps)
        e[1].record()
        for i, k in enumerate(ks):
            e[2 + 2 * i].record()
            self.arb.arb_count_async(o["ooff"], o["oidx"], k, total=self.totals[k], per_vertex=self.pvs.get(k),
                                     opts=self.opts[sname][k], ws=self.wss[k])
            e[3 + 2 * i].record()
        torch.cuda.synchronize()
        t_orient = e[0].elapsed_time(e[1]) / 1e3
        return t_orient, {k: e[2 + 2 * i].elapsed_time(e[3 + 2 * i]) / 1e3 for i, k in enumerate(ks)}

    def compare_schedules(self, main, ms_main, tot, steps, warmup):
        cmp = {main: ms_main}
        for sname in ("learned", "degree", "plain"):
            if sname not in cmp:
                ms_o, tot_o = self.timed(sname, steps, warmup)
                if tot_o != tot:
                    raise SystemExit(f"{self.name}: schedule {sname} changed the totals: {tot_o} vs {tot}")
                cmp[sname] = ms_o
        return {"ms_per_step": cmp, "learned_gain_vs_degree": cmp["degree"] / cmp["learned"],
                "learned_gain_vs_plain": cmp["plain"] / cmp["learned"]}


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-child":
        cpu_child(sys.argv[2], [int(x) for x in sys.argv[3].split(",")], int(sys.argv[4]))
        return
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "bench.py measures one GPU; runs on several GPUs are not implemented",
                          "n_gpus": a.gpus}))
        log("bench.py runs on exactly one GPU (--gpus 1): the counting path is not sharded across GPUs")
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2002_10047_amd import arb
    from paper_2002_10047_amd import graphgen as gg

    if a.only == "rmat26":
        n26, off26, idx26 = gg.rmat_cb_device(26, 1 << 30, seed=51)
        w26 = Workload(arb, torch, "rmat26", n26, off26, idx26, [4], a.eps, False, a, "rmat26", tune=False)
        w26.timed(a.schedule, a.steps, a.warmup)
        copy_calibration(a, torch)
        return
    if a.only == "rmat20":
        g = gg.config_graph("c2")
        off20, idx20 = arb.to_device_csr(g)
        w20 = Workload(arb, torch, "rmat20", g.n, off20, idx20, [3, 4, 5], a.eps, False, a, "rmat20")
        w20.timed(a.schedule, a.steps, a.warmup)
        copy_calibration(a, torch)
        return

    # ---------------------------------------------------------------- headline: 3-D RGG
    ks = [5, 6, 7]
    t0 = time.time()
    n, off, idx = gg.rgg_cb_device(1 << 24, 40.0, seed=52)
    torch.cuda.synchronize()
    log(f"3-D RGG: n={n} m={idx.numel() // 2} generated on the GPU in {time.time() - t0:.1f}s")
    hw = Workload(arb, torch, "rgg3d", n, off, idx, ks, a.eps, True, a, "rgg3d")
    main_name = a.schedule
    arb.arb_profile_enable(True)          # kernel timings cover the headline's timed steps only
    ms_step, tot = hw.timed(main_name, a.steps, a.warmup)
    prof = [e for e in arb.arb_profile_read() if not e["instrumented"]]
    arb.arb_profile_enable(False)
    cliques = sum(tot.values())
    exact = (golden("c5b") or {}).get("totals", {})
    out = {
        "metric": "k-cliques/s & oriented edges/s (exact), learned vs degree schedule, 1 GPU",
        "value": cliques / (ms_step / 1e3), "unit": "k-cliques/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "rgg3d_2^24_deg40_k567_per_vertex",
                   "graph": "3-D random geometric graph on the unit torus, 2^24 vertices, mean degree 40, "
                            "counter-based stream seed 52",
                   "n": n, "m": hw.m, "k": ks, "per_vertex": True, "eps": a.eps, "schedule": main_name,
                   "opts": {str(k): arb.opts_dict(hw.opts[main_name][k]) for k in ks},
                   "totals": {str(k): tot[k] for k in ks},
                   "totals_equal_oracle": ({str(k): tot[k] == exact[str(k)] for k in ks} if exact else None)},
    }
    if a.no_extras:
        copy_calibration(a, torch)
        print(json.dumps(out), flush=True)
        return
    out["schedules"] = hw.compare_schedules(main_name, ms_step, tot, a.steps, a.warmup)
    t_or, t_k = hw.phases(main_name)
    out["orient_s"] = t_or
    out["oriented_edges_per_s"] = hw.m / t_or
    out["per_k"] = {str(k): {"count_s": t_k[k], "cliques": tot[k], "cliques_per_s": tot[k] / t_k[k]} for k in ks}
    log(f"rgg3d orient {t_or * 1e3:.2f} ms ({hw.m / t_or:.3g} oriented edges/s); " +
        ", ".join(f"k={k}: {t_k[k] * 1e3:.2f} ms" for k in ks))
    rf, phase = roofline(arb, np, torch, hw.o, ks, True, hw.opts[main_name], prof, "rgg3d_k567_pv")
    out["roofline"] = rf
    for k, u in phase.items():
        t = t_k[k]
        out["per_k"][str(k)].update({"alu_Tops": u["alu"] / t / 1e12, "alu_frac": u["alu"] / t / 1e12 / PEAK_ALU_TOPS,
                                     "lds_GBs": u["lds"] / t / 1e9, "hbm_GBs": u["hbm"] / t / 1e9})
    del hw, off, idx
    torch.cuda.empty_cache()

    # ---------------------------------------------------------------- R-MAT scale 26, k = 4
    if not a.no_rmat26:
        t0 = time.time()
        n26, off26, idx26 = gg.rmat_cb_device(26, 1 << 30, seed=51)
        torch.cuda.synchronize()
        log(f"R-MAT 26: n={n26} m={idx26.numel() // 2} generated on the GPU in {time.time() - t0:.1f}s")
        # library defaults: a search on this graph takes several seconds per candidate
        w26 = Workload(arb, torch, "rmat26", n26, off26, idx26, [4], a.eps, False, a, "rmat26", tune=False)
        arb.arb_profile_enable(True)
        ms26, tot26 = w26.timed(main_name, 2, 1)
        prof26 = [e for e in arb.arb_profile_read() if not e["instrumented"]]
        arb.arb_profile_enable(False)
        sch = w26.compare_schedules(main_name, ms26, tot26, 2, 1)
        t_or, t_k = w26.phases(main_name)
        rf26, _ = roofline(arb, np, torch, w26.o, [4], False, w26.opts[main_name], prof26, "rmat26_k4")
        out["rmat26_k4"] = {"n": n26, "m": w26.m, "total": tot26[4], "orient_s": t_or,
                            "oriented_edges_per_s": w26.m / t_or, "count_s": t_k[4],
                            "cliques_per_s": tot26[4] / t_k[4], "step_ms": sch["ms_per_step"],
                            "learned_gain_vs_degree": sch["learned_gain_vs_degree"],
                            "learned_gain_vs_plain": sch["learned_gain_vs_plain"],
                            "opts": arb.opts_dict(w26.opts[main_name][4]), "roofline": rf26}
        log(f"rmat26 k=4: {out['rmat26_k4']}")
        del w26, off26, idx26
        torch.cuda.empty_cache()

    # ---------------------------------------------------------------- R-MAT scale 20, k = 3, 4, 5
    g = gg.config_graph("c2")
    off20, idx20 = arb.to_device_csr(g)
    w20 = Workload(arb, torch, "rmat20", g.n, off20, idx20, [3, 4, 5], a.eps, False, a, "rmat20")
    arb.arb_profile_enable(True)
    ms20, tot20 = w20.timed(main_name, a.steps, a.warmup)
    prof20 = [e for e in arb.arb_profile_read() if not e["instrumented"]]
    arb.arb_profile_enable(False)
    sch = w20.compare_schedules(main_name, ms20, tot20, a.steps, a.warmup)
    t_or, t_k = w20.phases(main_name)
    # every tier kernel's fractions side by side (the k = 5 tiers run concurrently, so a
    # kernel's own fraction understates the machine's), and the whole count of each k
    rf20, ph20 = roofline(arb, np, torch, w20.o, [3, 4, 5], False, w20.opts[main_name], prof20, "rmat20_k345")
    out["rmat20_k345"] = {"n": g.n, "m": g.m, "totals": {str(k): v for k, v in tot20.items()}, "orient_s": t_or,
                          "oriented_edges_per_s": g.m / t_or, "count_s": {str(k): t for k, t in t_k.items()},
                          "step_ms": sch["ms_per_step"], "value": sum(tot20.values()) / (ms20 / 1e3),
                          "learned_gain_vs_degree": sch["learned_gain_vs_degree"],
                          "learned_gain_vs_plain": sch["learned_gain_vs_plain"], "roofline": rf20,
                          "per_k_fracs": {str(k): {"alu": u["alu"] / t_k[k] / 1e12 / PEAK_ALU_TOPS,
                                                   "hbm": u["hbm"] / t_k[k] / 1e9 / PEAK_HBM_GBS}
                                          for k, u in ph20.items()}}

    if not a.no_studies:
        studies(arb, gg, torch, g, off20, idx20, w20, tot20, a, out)
    del w20

    # ---------------------------------------------------------------- CPU oracle baseline
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(ks, a.cpu_seconds, exact, n)
    copy_calibration(a, torch)
    print(json.dumps(out), flush=True)


def studies(arb, gg, torch, g, off, idx, w20, tot, a, out):
    """The paper's other rows on R-MAT 20: colorful sparsification (Sec. 3.3), the
    orderings of Sec. 5 and arb-approx-peel (Sec. 4.2)."""
    kx = max(w20.ks)
    approx = {}
    for c in (2, 4, 8):
        col = torch.from_numpy(gg.colors(g.n, c, 7)).cuda()
        torch.cuda.synchronize()
        t1 = time.time()
        soff, sidx = arb.arb_sparsify(off, idx, col)
        so = arb.arb_orient(soff, sidx, eps=a.eps)
        cnt = arb.arb_count(so["ooff"], so["oidx"], kx)
        dt = time.time() - t1
        est = arb.arb_colorful_estimate(cnt, c, kx)
        approx[str(c)] = {"k": kx, "seconds": dt, "kept_edges": int(sidx.numel() // 2), "count": cnt,
                          "estimate": est, "rel_error": (est - tot[kx]) / tot[kx] if tot[kx] else None}
    out["colorful_sparsification"] = approx
    study = {}
    for name, meth in (("peel", arb.ARB_ORIENT_PEEL), ("degree", arb.ARB_ORIENT_DEGREE),
                       ("goodrich_pszona", arb.ARB_ORIENT_GOODRICH_PSZONA), ("kcore", arb.ARB_ORIENT_KCORE)):
        arb.arb_orient_method(off, idx, meth, eps=a.eps)
        torch.cuda.synchronize()
        t1 = time.time()
        om = arb.arb_orient_method(off, idx, meth, eps=a.eps)
        torch.cuda.synchronize()
        t_or = time.time() - t1
        wsx = arb.CountWorkspace(om["ooff"], om["oidx"], kx)
        arb.arb_count(om["ooff"], om["oidx"], kx, ws=wsx)
        torch.cuda.synchronize()
        t1 = time.time()
        cnt = arb.arb_count(om["ooff"], om["oidx"], kx, ws=wsx)
        t_ct = time.time() - t1
        if cnt != tot[kx]:
            raise SystemExit(f"ordering {name} changed the k={kx} count")
        study[name] = {"orient_ms": t_or * 1e3, "rounds": int(om["stats"][0]), "max_outdeg": int(om["stats"][1]),
                       f"count_k{kx}_ms": t_ct * 1e3}
        del wsx
    out["orientation_study"] = study
    torch.cuda.synchronize()
    t1 = time.time()
    dens, rounds, _ = arb.arb_approx_peel(w20.o["ooff"], w20.o["oidx"], 3, 1.0)
    out["approx_peel"] = {"k": 3, "eps": 1.0, "seconds": time.time() - t1, "rounds": rounds, "density": dens}


if __name__ == "__main__":
    main()
