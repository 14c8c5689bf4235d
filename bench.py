#!/usr/bin/env python3
"""Throughput benchmark of the arb-count hot path on one MI355X.

Workload: R-MAT scale 20 (2^20 vertices, 2^24 edge samples, a,b,c,d = .57,.19,.19,.05,
seeded permutation, self-loops and duplicates removed), k = 3, 4, 5.

One step = the whole hot path on the resident graph: arb_orient (eps = 1) followed by
arb_count for k = 3, 4 and 5 (exact totals).  `value` = k-cliques counted per second of
step time (sum over the three k).  The JSON line also carries oriented edges/s, per-k
rates, the roofline of the dominant counting kernel and the CPU-oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--ks", default="3,4,5")
    ap.add_argument("--eps", type=float, default=1.0)
    ap.add_argument("--schedule", default="learned", choices=["plain", "persistent", "degree", "learned"])
    ap.add_argument("--no-tune", action="store_true", help="library default options, no autotuning")
    ap.add_argument("--retune", action="store_true", help="run the autotuner even if options are cached")
    ap.add_argument("--tune-cache", default="", help="tuned-options cache file (default: the package's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="only the timed steps (profiling runs)")
    ap.add_argument("--no-studies", action="store_true",
                    help="skip the studies after the roofline (sparsification, orderings, peeling), so that a "
                         "kernel trace of the run holds only the launches the roofline averages")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="after the run, copy a buffer of this size once (counter calibration)")
    return ap.parse_args()


def algorithmic_units(arb, o, ks, np):
    """Per-root algorithmic units from the instrumented count: gather words and the
    numbers c_j(v) of j-cliques inside G[N+(v)] (j <= k-2)."""
    import torch
    ooff = o["ooff"].cpu().numpy()
    oidx = o["oidx"].cpu().numpy()
    n = len(ooff) - 1
    d = np.diff(ooff)
    rows = np.repeat(np.arange(n), d)
    gather = np.bincount(rows, weights=d[oidx].astype(np.float64), minlength=n).astype(np.int64)
    W = (d + 31) // 32
    nodes = {}
    for k in sorted(set(ks) | {k - 1 for k in ks if k >= 4} | {3}):
        work = torch.empty(n, dtype=torch.int64, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, work=work)
        torch.cuda.synchronize()
        wk = work.cpu().numpy()
        live = d >= k - 1
        nd = np.zeros(n, np.int64)
        nd[live] = (wk[live] - gather[live]) // W[live]
        nodes[k] = nd
    return d, W, gather, nodes


def cpu_child(path, k, budget, cores):
    """Child process: time the CPU oracle on a strided sample of roots (its degree order,
    positions p with p % stride == stride // 2), shrinking the stride until the sample
    takes about `budget` seconds.  Prints one JSON line."""
    import numpy as np
    import oracle
    from paper_2002_10047_amd import graphgen as gg
    z = np.load(path)
    g = gg.Graph(int(z["n"]), z["offsets"], z["indices"])
    stride = 1 << 16
    while True:
        t1 = time.time()
        c = oracle.count(g, k, nthreads=cores, stride=stride, phase=stride // 2)
        dt = time.time() - t1
        print(json.dumps({"k": k, "stride": stride, "count": c, "seconds": dt}), flush=True)
        if dt >= budget / 4 or stride == 1:
            break
        stride = max(1, stride // 4)


def cpu_baseline(g, ks, seconds):
    import subprocess
    import tempfile
    import numpy as np
    cores = min(16, os.cpu_count() or 1)
    budget = seconds / len(ks)
    with tempfile.TemporaryDirectory() as td:
        path = os.path.join(td, "g.npz")
        np.savez(path, n=g.n, offsets=g.offsets, indices=g.indices)
        samp, cnt_x, t_x = [], 0.0, 0.0
        for k in ks:
            last = None
            try:
                r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-child", path, str(k),
                                    str(budget), str(cores)], capture_output=True, text=True,
                                   timeout=max(30.0, 6 * budget))
                lines = [l for l in r.stdout.splitlines() if l.startswith("{")]
                last = json.loads(lines[-1]) if lines else None
            except subprocess.TimeoutExpired as e:
                lines = [l for l in (e.stdout or b"").decode().splitlines() if l.startswith("{")]
                last = json.loads(lines[-1]) if lines else None
            if not last or last["seconds"] <= 0:
                continue
            cnt_x += last["count"] * last["stride"]
            t_x += last["seconds"] * last["stride"]
            samp.append(f"k={k}: roots at positions p % {last['stride']} == {last['stride'] // 2} of the oracle's "
                        f"degree order, {last['count']} cliques in {last['seconds']:.2f}s")
            log(f"cpu oracle {samp[-1]}")
    if t_x <= 0:
        return None
    return {"value": cnt_x / t_x, "unit": "k-cliques/s", "cores": cores, "kind": "oracle",
            "sample": "Chiba-Nishizeki oracle (OpenMP over roots) on the same graph; per k a strided root "
                      "sample scaled by its stride, rate = sum(count*stride)/sum(seconds*stride); " + "; ".join(samp)}


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
    for f in ("count_kernels.h", "count.hip"):
        with open(os.path.join(ROOT, "paper_2002_10047_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was
    taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", "traffic_counters.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        t = json.load(f)
    if t.get("source_hash") != kernel_source_hash():
        return None
    e = t.get("kernels", {}).get(kernel)
    return None if e is None else e.get("hbm_bytes_per_launch")


def tier_of(d):
    import numpy as np
    b = np.array([64, 128, 256, 384, 512, 768])
    return np.searchsorted(b, d, side="left")


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--cpu-child":
        cpu_child(sys.argv[2], int(sys.argv[3]), float(sys.argv[4]), int(sys.argv[5]))
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

    ks = [int(x) for x in a.ks.split(",")]
    arb.arb_profile_enable(True)
    t0 = time.time()
    g = gg.config_graph("c2")
    log(f"graph: n={g.n} m={g.m} generated in {time.time() - t0:.1f}s")
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx, eps=a.eps)
    wss = {k: arb.CountWorkspace(o["ooff"], o["oidx"], k) for k in ks}
    totals = {k: torch.empty(1, dtype=torch.int64, device="cuda") for k in ks}
    from paper_2002_10047_amd import learn
    weights = {k: learn.load_weights(k) for k in ks}
    missing = [k for k in ks if weights[k] is None]
    if missing:
        raise SystemExit(f"no trained cost model for k={missing}: run python -m paper_2002_10047_amd.train_cost")
    feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])

    # ---------------------------------------------------------------- tuning (untimed)
    schedules = {}
    t_tune = time.time()
    from paper_2002_10047_amd import tuning
    cache = a.tune_cache or tuning.CACHE
    for name in ("degree", "learned"):
        per_k = {}
        for k in ks:
            if a.no_tune:
                op = arb.count_opts(schedule=tuning.SCHEDULES[name], mlp_weights=weights[k] if name == "learned" else None,
                                    features=feat if name == "learned" else None)
            else:
                op, _ = tuning.tuned_opts(o["ooff"], o["oidx"], k, name, mlp_weights=weights[k] if name == "learned" else None,
                                          features=feat if name == "learned" else None, ws=wss[k], retune=a.retune,
                                          path=cache, log=log)
            per_k[k] = op
        schedules[name] = per_k
    schedules["plain"] = {k: arb.count_opts(schedule=arb.ARB_SCHED_PLAIN) for k in ks}
    log(f"tuning took {time.time() - t_tune:.1f}s")
    arb.arb_profile_enable(True)      # the kernel timings cover the timed steps only, not tuning

    def step(name):
        oo = arb.arb_orient(off, idx, eps=a.eps)
        if name == "learned":
            f = arb.arb_features(oo["ooff"], oo["oidx"], oo["round"], oo["rank"])
            for k in ks:
                schedules[name][k].features = f.data_ptr()
                schedules[name][k]._keep = (weights[k], f)
        for k in ks:
            arb.arb_count_async(oo["ooff"], oo["oidx"], k, total=totals[k], opts=schedules[name][k], ws=wss[k])
        return oo

    def timed(name):
        for i in range(a.warmup):
            step(name)
            torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record()
        for i in range(a.steps):
            step(name)
        ev1.record()
        torch.cuda.synchronize()
        ms = ev0.elapsed_time(ev1) / a.steps
        tot = {k: int(totals[k].cpu().numpy().view(np.uint64)[0]) for k in ks}
        log(f"{name}: {ms:.3f} ms/step over {a.steps} steps, totals {tot}")
        return ms, tot

    main_name = a.schedule if a.schedule != "persistent" else "degree"
    ms_step, tot = timed(main_name)
    cliques = sum(tot.values())
    value = cliques / (ms_step / 1e3)
    out = {
        "metric": "k-cliques/s & oriented edges/s (exact), learned vs degree schedule, 1 GPU",
        "value": value, "unit": "k-cliques/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u32", "data": "synthetic",
        "config": {"workload": "rmat20_k345", "graph": "R-MAT scale 20, 2^24 samples, a=.57 b=.19 c=.19 d=.05, "
                   "seed 2, deduped", "n": g.n, "m": g.m, "k": ks, "eps": a.eps, "schedule": main_name,
                   "opts": {str(k): arb.opts_dict(schedules[main_name][k]) for k in ks},
                   "totals": {str(k): tot[k] for k in ks}},
    }
    if not a.no_extras:
        cmp = {main_name: ms_step}
        for name in ("learned", "degree", "plain"):
            if name not in cmp:
                ms_o, tot_o = timed(name)
                if tot_o != tot:
                    raise SystemExit(f"schedule {name} changed the totals: {tot_o} vs {tot}")
                cmp[name] = ms_o
        out["schedules_ms_per_step"] = cmp
        out["learned_gain_vs_degree"] = cmp["degree"] / cmp["learned"]
        out["learned_gain_vs_plain"] = cmp["plain"] / cmp["learned"]
        opts = schedules[main_name][ks[0]]
    if a.no_extras:
        copy_calibration(a, torch)
        print(json.dumps(out), flush=True)
        return

    # ---------------------------------------------------------------- phase breakdown
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2 + 2 * len(ks))]
    torch.cuda.synchronize()
    e[0].record()
    o = arb.arb_orient(off, idx, eps=a.eps)
    e[1].record()
    for i, k in enumerate(ks):
        e[2 + 2 * i].record()
        arb.arb_count_async(o["ooff"], o["oidx"], k, total=totals[k], opts=schedules[main_name][k], ws=wss[k])
        e[3 + 2 * i].record()
    torch.cuda.synchronize()
    t_orient = e[0].elapsed_time(e[1]) / 1e3
    per_k = {}
    for i, k in enumerate(ks):
        tk = e[2 + 2 * i].elapsed_time(e[3 + 2 * i]) / 1e3
        per_k[str(k)] = {"count_s": tk, "cliques": tot[k], "cliques_per_s": tot[k] / tk}
    out["oriented_edges_per_s"] = g.m / t_orient
    out["orient_s"] = t_orient
    out["per_k"] = per_k
    log(f"orient {t_orient * 1e3:.3f} ms; per k: " +
        ", ".join(f"k={k}: {v['count_s'] * 1e3:.3f} ms" for k, v in per_k.items()))

    # ---------------------------------------------------------------- roofline
    # every counting-kernel launch of this run was timed with HIP events on its own
    # stream; a kernel symbol k_count<W, depth, 0, 0> serves tier W and depth max(1, k-3)
    prof = [e for e in arb.arb_profile_read() if not e["per_vertex"] and not e["instrumented"]]
    arb.arb_profile_enable(False)
    d, W, gather, nodes = algorithmic_units(arb, o, ks, np)
    tw = [2, 4, 8, 12, 16, 24]
    per_sym = {}
    phase_units = {}            # per k: algorithmic units of one count (all tiers)
    peaks = measure_peaks(torch)
    peak_lds = max(SPEC_LDS_GBS, peaks["lds_read_GBs"] or 0.0)
    log(f"probes: LDS read {peaks['lds_read_GBs']:.0f} GB/s, device copy {peaks['copy_GBs']:.0f} GB/s "
        f"(LDS peak used {peak_lds:.0f} GB/s)")
    for e in prof:
        k, ti = e["k"], e["tier"]
        live = d >= k - 1
        td = tier_of(d)
        if k >= 5:
            td = np.minimum(td, 5)       # above 768 out-neighbours: per-out-neighbour items in tier 5
        sel = live & (td == ti)
        hbm_bytes = float(4 * (d[sel] + 4 * d[sel] + gather[sel]).sum() + 16 * sel.sum())
        alu_ops = lds_bytes = 0.0
        if k >= 4:
            ck2 = nodes[k][sel] - nodes[k - 1][sel]          # c_{k-2}(v)
            deep = nodes[k][sel] - d[sel]                    # sum_{j=2}^{k-2} c_j(v)
            # every node of depth >= 2 ANDs W words; nodes of depth k-2 also popcount them
            alu_ops = float((W[sel] * (deep + ck2)).sum())
            # bit rows built (d), a row read and I' written per internal node (depth
            # 1..k-3), a row read per node of depth k-2: 4 W (d + 2 sum_{j<=k-3} c_j + c_{k-2})
            lds_bytes = float((4 * W[sel] * (d[sel] + nodes[k - 1][sel] + nodes[k][sel])).sum())
        sym = f"k_count<{tw[ti]},{max(1, k - 3)},0,0>" if ti < len(tw) else "k_count_big<0,0>"
        s_ = per_sym.setdefault(sym, dict(launches=0, ms=0.0, hbm=0.0, alu=0.0, lds=0.0, parts=[]))
        s_["launches"] += e["launches"]
        s_["ms"] += e["total_ms"]
        s_["hbm"] += e["launches"] * hbm_bytes
        s_["alu"] += e["launches"] * alu_ops
        s_["lds"] += e["launches"] * lds_bytes
        pk = phase_units.setdefault(k, dict(alu=0.0, lds=0.0, hbm=0.0))
        pk["alu"] += alu_ops
        pk["lds"] += lds_bytes
        pk["hbm"] += hbm_bytes
        s_["parts"].append(f"k={k}: {e['launches']} launches, {e['total_ms'] / e['launches']:.3f} ms avg")
    best = None
    for sym, v in sorted(per_sym.items()):
        sec = v["ms"] / 1e3
        hbm = v["hbm"] / sec / 1e9
        alu = v["alu"] / sec / 1e12
        lds = v["lds"] / sec / 1e9
        log(f"  {sym}: {v['launches']} launches, avg {v['ms'] / v['launches']:.3f} ms ({'; '.join(v['parts'])}), "
            f"algorithmic {hbm:.0f} GB/s ({hbm / PEAK_HBM_GBS:.2%} of HBM), {alu:.2f} Tops ({alu / PEAK_ALU_TOPS:.2%} "
            f"of ALU), LDS {lds:.0f} GB/s ({lds / peak_lds:.2%})")
        if best is None or v["ms"] > best[1]["ms"]:
            best = (sym, v, hbm, alu, lds)
    if best:
        sym, v, hbm, alu, lds = best
        fr = {"hbm": hbm / PEAK_HBM_GBS, "alu": alu / PEAK_ALU_TOPS, "lds": lds / peak_lds}
        bound = max(fr, key=fr.get)
        unit = {"hbm": ("GB/s", hbm, PEAK_HBM_GBS), "alu": ("Tops/s", alu, PEAK_ALU_TOPS),
                "lds": ("GB/s", lds, peak_lds)}[bound]
        out["roofline"] = {"bound": bound, "achieved": unit[1], "peak": unit[2], "unit": unit[0], "frac": fr[bound]}
        out["roofline"]["traffic"] = measured_traffic(sym)
        out["roofline"]["kernel"] = sym
        out["roofline"]["launches"] = v["launches"]
        out["roofline"]["launch_ms"] = v["ms"] / v["launches"]
        out["roofline"]["algorithmic_per_launch"] = {"hbm": v["hbm"], "alu": v["alu"], "lds": v["lds"]}[bound] / \
            v["launches"]
        out["roofline"]["fracs"] = fr
        out["roofline"]["lds_words_per_s"] = lds * 1e9 / 4
        out["roofline"]["peaks_measured"] = peaks
    # whole count of each k (all tier kernels, concurrent): algorithmic rates over its time
    for k, u in phase_units.items():
        if str(k) in per_k:
            t = per_k[str(k)]["count_s"]
            per_k[str(k)]["alu_Tops"] = u["alu"] / t / 1e12
            per_k[str(k)]["alu_frac"] = u["alu"] / t / 1e12 / PEAK_ALU_TOPS
            per_k[str(k)]["lds_GBs"] = u["lds"] / t / 1e9
            per_k[str(k)]["hbm_GBs"] = u["hbm"] / t / 1e9

    if a.no_studies:
        if not a.no_cpu_baseline:
            out["cpu_baseline"] = cpu_baseline(g, ks, a.cpu_seconds)
        copy_calibration(a, torch)
        print(json.dumps(out), flush=True)
        return

    # ---------------------------------------------------------------- colorful sparsification
    # approximate counts (Sec. 3.3): sparsify with c colours, orient and count the sparsified
    # graph; time of the three (wall clock, synchronised) and the estimate's relative error
    approx = {}
    kx = max(ks)
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

    # ---------------------------------------------------------------- orientation study
    # the orderings the paper compares (Sec. 5): orientation time, largest out-degree and
    # the count of the largest k on each (degree schedule, library defaults)
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

    # ---------------------------------------------------------------- approximate peeling
    # arb-approx-peel (Sec. 4.2) for k = 3 on the same graph
    torch.cuda.synchronize()
    t1 = time.time()
    dens, rounds, _ = arb.arb_approx_peel(o["ooff"], o["oidx"], 3, 1.0)
    out["approx_peel"] = {"k": 3, "eps": 1.0, "seconds": time.time() - t1, "rounds": rounds, "density": dens}

    # ---------------------------------------------------------------- CPU oracle baseline
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, ks, a.cpu_seconds)
    copy_calibration(a, torch)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
