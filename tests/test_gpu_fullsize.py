"""Parity at the full size of the R-MAT scale-20 workload (2^20 vertices, 15.7M edges) in
the launch configuration bench.py times: learned schedule, tuned options from the cache,
concurrent tier kernels.  The oracle cannot count k = 4, 5 on the whole graph in test time,
so it checks sampled outputs one by one -- per-root counts (the (k-1)-cliques of
G[N+(v)] on the GPU's own orientation, heaviest roots included) and per-vertex counts
(from each sampled vertex's neighbourhood) -- plus properties that hold at any size:
per-root counts sum to the total, per-vertex counts to k times the total.  The k = 3
total is checked whole."""
import sys

import numpy as np
import pytest
import torch

from paper_2002_10047_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def arb():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_10047_amd.arb as arb
    return arb


@pytest.fixture(scope="module")
def c2(arb):
    say("generating R-MAT scale 20")
    g = gg.config_graph("c2")
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx, eps=1.0)
    feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])
    host = dict(ooff=o["ooff"].cpu().numpy(), oidx=o["oidx"].cpu().numpy(), rank=o["rank"].cpu().numpy())
    return g, o, feat, host


def bench_opts(arb, o, feat, k, ws):
    from paper_2002_10047_amd import learn, tuning
    w = learn.load_weights(k)
    assert w is not None, f"no trained cost model for k={k}"
    op, _ = tuning.tuned_opts(o["ooff"], o["oidx"], k, "learned", mlp_weights=w, features=feat, ws=ws)
    op._keep = (w, feat)
    return op


def sample_roots(d, k, rng):
    live = np.nonzero(d >= k - 1)[0]
    heavy = np.argsort(-d)[: (20 if k >= 5 else 100)]
    bounds = [0, 64, 128, 256, 384, 512, 768]
    per_tier = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        t = live[(d[live] > lo) & (d[live] <= hi)]
        if t.size:
            per_tier.append(rng.choice(t, min(t.size, 200 if hi <= 256 else 40), replace=False))
    return np.unique(np.concatenate([heavy, *per_tier, rng.choice(live, 1000, replace=False)]))


@pytest.mark.parametrize("k", [3, 4, 5])
def test_full_c2_per_root_sampled(arb, orc, c2, k):
    g, o, feat, host = c2
    n = g.n
    ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
    per_root = torch.empty(n, dtype=torch.int64, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, opts=bench_opts(arb, o, feat, k, ws),
                        ws=ws)
    torch.cuda.synchronize()
    pr = arb.u64_numpy(per_root)
    t = int(arb.u64_numpy(total)[0])
    assert int(pr.sum(dtype=np.uint64)) == t
    d = np.diff(host["ooff"])
    roots = sample_roots(d, k, np.random.default_rng(100 + k))
    say("k", k, "total", t, "checking", roots.size, "roots; max d+ among them", int(d[roots].max()))
    ref = orc.local_cliques_roots(n, host["ooff"], host["oidx"], k - 1, roots, nthreads=16)
    assert np.array_equal(pr[roots], ref[:, k - 2])
    if k == 3:
        assert t == orc.count(g, 3, nthreads=16)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_full_c2_per_vertex_sampled(arb, orc, c2, k):
    g, o, feat, host = c2
    deg = np.diff(g.offsets)
    cap = 3000 if k <= 4 else 500
    ok = np.nonzero(deg <= cap)[0]
    rng = np.random.default_rng(200 + k)
    verts = np.unique(np.concatenate([rng.choice(ok, 300, replace=False), ok[np.argsort(-deg[ok])[:20]]]))
    ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
    op = bench_opts(arb, o, feat, k, ws)
    t, pv_rank = arb.arb_count(o["ooff"], o["oidx"], k, per_vertex=True, opts=op, ws=ws)
    assert int(pv_rank.sum(dtype=np.uint64)) == (k * t) % (1 << 64)
    pv = pv_rank[host["rank"]]                      # back to the generator's vertex ids
    say("k", k, "per-vertex: checking", verts.size, "vertices of degree <=", cap)
    ref = orc.vertex_cliques(g, k, verts, nthreads=16)
    assert np.array_equal(pv[verts], ref)


def csr_digest(off, idx) -> str:
    import hashlib
    h = hashlib.sha256()
    h.update(off.cpu().numpy().astype(np.int64).tobytes())
    h.update(idx.cpu().numpy().astype(np.int32).tobytes())
    return h.hexdigest()


def golden_totals(name):
    import json
    import os
    p = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_totals.json")
    with open(p) as f:
        return json.load(f)[name]


def test_full_c2_totals_golden(arb, c2):
    # k = 3, 4, 5 totals of the whole graph against the oracle's (tests/golden/make_fullsize.py)
    g, o, feat, host = c2
    ref = golden_totals("c2")
    assert (ref["n"], ref["m"]) == (g.n, g.m)
    ref["totals"].update(golden_totals("c2k5")["totals"])
    for k in (3, 4, 5):
        ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
        assert arb.arb_count(o["ooff"], o["oidx"], k, opts=bench_opts(arb, o, feat, k, ws), ws=ws) == \
            ref["totals"][str(k)]


@pytest.fixture(scope="module")
def c3(arb):
    say("generating Chung-Lu n=2^22 with 1000 planted communities")
    g = gg.config_graph("c3")
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx, eps=1.0)
    host = dict(ooff=o["ooff"].cpu().numpy(), oidx=o["oidx"].cpu().numpy(), rank=o["rank"].cpu().numpy())
    return g, o, host


@pytest.mark.parametrize("k", [6, 7, 8])
def test_full_c3_totals_and_samples(arb, orc, c3, k):
    """Chung-Lu 2^22 vertices (exponent 2.1, 2^26 pairs, weights capped at 4000) with 1000
    planted communities of 40-80 vertices at edge probability 1/2: the deep-recursion
    workload.  Totals against the oracle's; per-root counts of the heaviest and of random
    roots, and per-vertex counts of community-sized neighbourhoods, one by one."""
    g, o, host = c3
    ref = golden_totals("c3")
    assert (ref["n"], ref["m"]) == (g.n, g.m)
    n = g.n
    ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
    per_root = torch.empty(n, dtype=torch.int64, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, ws=ws)
    torch.cuda.synchronize()
    t = int(arb.u64_numpy(total)[0])
    assert t == ref["totals"][str(k)]
    pr = arb.u64_numpy(per_root)
    assert int(pr.sum(dtype=np.uint64)) == t
    d = np.diff(host["ooff"])
    roots = sample_roots(d, k, np.random.default_rng(300 + k))
    roots = np.unique(np.concatenate([roots, np.nonzero(pr)[0][:2000]]))    # roots that own cliques
    say("k", k, "total", t, "checking", roots.size, "roots")
    lc = orc.local_cliques_roots(n, host["ooff"], host["oidx"], k - 1, roots, nthreads=16)
    assert np.array_equal(pr[roots], lc[:, k - 2])
    tp, pv_rank = arb.arb_count(o["ooff"], o["oidx"], k, per_vertex=True, ws=ws)
    assert tp == t and int(pv_rank.sum(dtype=np.uint64)) == (k * t) % (1 << 64)
    pv = pv_rank[host["rank"]]
    deg = np.diff(g.offsets)
    rng = np.random.default_rng(400 + k)
    inside = np.nonzero(pv)[0]
    verts = np.unique(np.concatenate([rng.choice(np.nonzero(deg <= 300)[0], 300, replace=False),
                                      inside[deg[inside] <= 300][:300]]))
    assert np.array_equal(pv[verts], orc.vertex_cliques(g, k, verts, nthreads=16))


def test_full_c4_batch_learned_in_one_graph(arb):
    """The batch of 256 graphs of uneven size (10^4..5*10^5 edges; G(n,p), R-MAT scales
    12-18, 2-D random geometric) as one disjoint union: per-graph orientation, features,
    and learned-schedule counts for k = 4, 5 captured in one hipGraph; every graph's
    total against the oracle's, eagerly and on replays."""
    from paper_2002_10047_amd import learn
    say("generating the 256-graph batch")
    gs = gg.batch_mix(256)
    ref = golden_totals("c4")
    assert ref["n"] == [g.n for g in gs] and ref["m"] == [g.m for g in gs]
    u, vo_h = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    vo = torch.from_numpy(vo_h).cuda()
    max_n = int(np.diff(vo_h).max())
    G = len(gs)
    ks = (4, 5)
    o = arb.arb_orient_batch(off, idx, vo, max_graph_n=max_n, validate=True)
    w = {k: learn.load_weights(k) for k in ks}
    ws = {k: arb._ws(arb.arb_count_batch_workspace(u.n, u.m, k, G), "cuda") for k in ks}
    tots = {k: torch.empty(G, dtype=torch.int64, device="cuda") for k in ks}

    def pipeline(stream=None):
        og = arb.arb_orient_batch(off, idx, vo, max_graph_n=max_n, stream=stream)
        f = arb.arb_features(og["ooff"], og["oidx"], og["round"], og["rank"], stream=stream)
        for k in ks:
            op = arb.count_opts(schedule=arb.ARB_SCHED_LEARNED, mlp_weights=w[k], features=f)
            arb.arb_count_batch_async(og["ooff"], og["oidx"], vo, k, totals=tots[k], opts=op, ws=ws[k],
                                      stream=stream)
        return og, f

    keep = pipeline()
    torch.cuda.synchronize()
    for k in ks:
        assert [int(x) for x in arb.u64_numpy(tots[k])] == ref["totals"][str(k)], k
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        keep = pipeline(torch.cuda.current_stream())
    for rep in range(2):
        for k in ks:
            tots[k].fill_(0)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in ks:
            assert [int(x) for x in arb.u64_numpy(tots[k])] == ref["totals"][str(k)], (k, rep)
    del keep


def _sample_and_check_roots(arb, orc, n, o, pr, k, rng, heavy=30, per_tier=150, rand=1000):
    ooff = o["ooff"].cpu().numpy()
    oidx = o["oidx"].cpu().numpy()
    d = np.diff(ooff)
    live = np.nonzero(d >= k - 1)[0]
    pick = [np.argsort(-d)[:heavy], rng.choice(live, min(rand, live.size), replace=False)]
    for lo, hi in zip([0, 64, 128, 256, 384, 512, 768], [64, 128, 256, 384, 512, 768, 1 << 40]):
        t = live[(d[live] > lo) & (d[live] <= hi)]
        if t.size:
            pick.append(rng.choice(t, min(t.size, per_tier), replace=False))
    roots = np.unique(np.concatenate(pick))
    say("k", k, "checking", roots.size, "roots, max d+", int(d[roots].max()))
    lc = orc.local_cliques_roots(n, ooff, oidx, k - 1, roots, nthreads=16)
    assert np.array_equal(pr[roots], lc[:, k - 2])


def _orientation_properties(arb, o, n, eps=1.0):
    import math
    rank = o["rank"]
    assert torch.equal(torch.sort(rank)[0], torch.arange(n, dtype=rank.dtype, device=rank.device))
    assert arb.arb_check_oriented(o["ooff"], o["oidx"]) == 0
    rounds = int(o["stats"][0])
    assert 1 <= rounds <= math.ceil(math.log(n) / math.log(2.0 + eps))
    thr = o["stats"][2:2 + rounds]
    dplus = o["ooff"][1:] - o["ooff"][:-1]                 # rank space
    assert bool((dplus[rank.long()] <= thr[o["round"].long()]).all())


def test_full_c5a_rmat26_k4(arb, orc):
    """R-MAT scale 26 (2^30 samples, 2^26 vertices, ~1.05 billion edges, built on the GPU
    from the counter-based stream): orientation invariants at full size, k = 4 total =
    sum of per-root counts (the whole-graph oracle count is hours of host time), per-root
    counts of the heaviest roots (2926 out-neighbours: the big-root path) and of every
    tier against the oracle, per-vertex counts of sampled vertices."""
    say("generating R-MAT scale 26 on the GPU")
    n, off, idx = gg.rmat_cb_device(26, 1 << 30, seed=51)
    assert arb.arb_validate(off, idx) == 0
    o = arb.arb_orient(off, idx, eps=1.0)
    _orientation_properties(arb, o, n)
    k = 4
    ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
    per_root = torch.empty(n, dtype=torch.int64, device="cuda")
    total = torch.empty(1, dtype=torch.int64, device="cuda")
    arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, ws=ws)
    torch.cuda.synchronize()
    t = int(arb.u64_numpy(total)[0])
    pr = arb.u64_numpy(per_root)
    del per_root
    assert int(pr.sum(dtype=np.uint64)) == t
    _sample_and_check_roots(arb, orc, n, o, pr, k, np.random.default_rng(51))
    tp, pv_rank = arb.arb_count(o["ooff"], o["oidx"], k, per_vertex=True, ws=ws)
    assert tp == t and int(pv_rank.sum(dtype=np.uint64)) == (4 * t) % (1 << 64)
    pv = pv_rank[o["rank"].cpu().numpy()]
    del pv_rank
    # vertices whose own and whose neighbours' degrees keep the oracle's merges short
    deg = (off[1:] - off[:-1])
    nbr_max = torch.zeros(n, dtype=torch.int64, device="cuda")
    rows = torch.repeat_interleave(torch.arange(n, device="cuda"), deg)
    nbr_max.scatter_reduce_(0, rows, deg[idx.long()], reduce="amax")
    del rows
    ok = torch.nonzero((deg >= 3) & (deg <= 1000) & (nbr_max <= 20000)).squeeze(1).cpu().numpy()
    verts = np.random.default_rng(52).choice(ok, 300, replace=False)
    g = gg.Graph(n, off.cpu().numpy(), idx.cpu().numpy())
    assert np.array_equal(pv[verts], orc.vertex_cliques(g, k, verts, nthreads=16))


def test_full_c5b_rgg3d(arb, orc):
    """3-D random geometric graph, 2^24 points on the unit torus, mean degree 40 (~335M
    edges, built on the GPU from the counter-based stream, byte-identical to the host's
    build): k = 5, 6, 7 totals against the oracle's, with per-vertex counts; per-root
    and per-vertex counts of sampled roots / vertices against the oracle; sums against
    the totals."""
    say("generating the 3-D random geometric graph on the GPU")
    n, off, idx = gg.rgg_cb_device(1 << 24, 40.0, seed=52)
    ref = golden_totals("c5b")
    assert (n, idx.numel() // 2) == (ref["n"], ref["m"])
    assert csr_digest(off, idx) == ref["sha256"]          # the graph the oracle counted
    assert arb.arb_validate(off, idx) == 0
    o = arb.arb_orient(off, idx, eps=1.0)
    _orientation_properties(arb, o, n)
    g = gg.Graph(n, off.cpu().numpy(), idx.cpu().numpy())
    rank = o["rank"].cpu().numpy()
    for k in (5, 6, 7):
        ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
        per_root = torch.empty(n, dtype=torch.int64, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, ws=ws)
        torch.cuda.synchronize()
        t = int(arb.u64_numpy(total)[0])
        pr = arb.u64_numpy(per_root)
        del per_root
        assert int(pr.sum(dtype=np.uint64)) == t
        assert t == ref["totals"][str(k)], k
        _sample_and_check_roots(arb, orc, n, o, pr, k, np.random.default_rng(60 + k), rand=500)
        tp, pv_rank = arb.arb_count(o["ooff"], o["oidx"], k, per_vertex=True, ws=ws)
        assert tp == t and int(pv_rank.sum(dtype=np.uint64)) == (k * t) % (1 << 64)
        verts = np.random.default_rng(70 + k).choice(n, 300, replace=False)
        assert np.array_equal(pv_rank[rank][verts], orc.vertex_cliques(g, k, verts, nthreads=16)), k
        say("k", k, "total", t)
