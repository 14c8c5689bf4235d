"""Batches of graphs as one disjoint union: arb_orient_batch peels every graph with its own
thresholds, so each graph's orientation must be byte-identical to the oracle's
orientation of that graph alone (shifted by its first vertex); arb_count_batch_async gives
per-graph totals from the contiguous rank ranges.  The whole pipeline (orientation and
counts for k = 4, 5) is captured in one hipGraph and replayed."""
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


def small_batch():
    gs = gg.batch_mix(10, m_lo=2e3, m_hi=3e4, seed_base=700)
    gs += [gg.empty(1), gg.complete(12), gg.turan(30, 5), gg.empty(4), gg.star(9), gg.gnp(300, 0.2, 9)]
    return gs


def oracle_batch_orient(orc, gs, eps):
    parts = dict(ooff=[np.zeros(1, np.int64)], oidx=[], rank=[], round=[], dap=[])
    base_v, base_a = 0, 0
    for g in gs:
        r = orc.orient(g, eps)
        parts["ooff"].append(r["ooff"][1:] + base_a)
        parts["oidx"].append(r["oidx"] + base_v)
        parts["rank"].append(r["rank"] + base_v)
        parts["round"].append(r["round"])
        parts["dap"].append(r["deg_at_peel"])
        base_v += g.n
        base_a += g.m
    return {k: np.concatenate(v) for k, v in parts.items()}


@pytest.mark.parametrize("eps", [1.0, 0.5, 2.0])
def test_batch_orientation_equals_separate_runs(arb, orc, eps):
    gs = small_batch()
    u, vo = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    o = arb.arb_orient_batch(off, idx, vo, eps=eps, validate=True)
    ref = oracle_batch_orient(orc, gs, eps)
    assert np.array_equal(o["ooff"].cpu().numpy(), ref["ooff"])
    assert np.array_equal(o["oidx"].cpu().numpy(), ref["oidx"])
    assert np.array_equal(o["rank"].cpu().numpy(), ref["rank"])
    assert np.array_equal(o["round"].cpu().numpy(), ref["round"])
    assert np.array_equal(o["deg_at_peel"].cpu().numpy(), ref["dap"])
    # a batch of one graph is arb_orient
    g = gs[0]
    off1, idx1 = arb.to_device_csr(g)
    a = arb.arb_orient(off1, idx1, eps=eps)
    b = arb.arb_orient_batch(off1, idx1, np.array([0, g.n]), eps=eps)
    for key in ("ooff", "oidx", "rank", "round", "deg_at_peel"):
        assert torch.equal(a[key], b[key]), key


def test_batch_rejects_bad_ranges_and_cross_edges(arb):
    gs = [gg.complete(6), gg.cycle(5)]
    u, vo = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    for bad in (np.array([0, 7, 11]), np.array([0, 6, 10]), np.array([1, 6, 11])):
        with pytest.raises(RuntimeError):
            arb.arb_orient_batch(off, idx, bad, validate=True)
    assert arb.arb_last_error() == arb.ARB_EGRAPH


def test_batch_counts_and_per_vertex(arb, orc):
    gs = small_batch()
    u, vo = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    o = arb.arb_orient_batch(off, idx, vo, validate=True)
    rank = o["rank"].cpu().numpy()
    for k in (3, 4, 5, 6):
        say("batch k", k)
        refs = [orc.count(g, k, per_vertex=True, nthreads=8) for g in gs]
        pv = torch.empty(u.n, dtype=torch.int64, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        tots = arb.arb_count_batch_async(o["ooff"], o["oidx"], o["vo"], k, total=total, per_vertex=pv)
        torch.cuda.synchronize()
        assert [int(x) for x in arb.u64_numpy(tots)] == [r[0] for r in refs]
        assert int(arb.u64_numpy(total)[0]) == sum(r[0] for r in refs)
        assert np.array_equal(arb.u64_numpy(pv)[rank], np.concatenate([r[1] for r in refs]))


def test_batch_pipeline_in_one_graph(arb, orc):
    gs = gg.batch_mix(24, m_lo=2e3, m_hi=4e4, seed_base=1300)
    u, vo_h = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    vo = torch.from_numpy(vo_h).cuda()
    max_n = int(np.diff(vo_h).max())
    refs = {k: [orc.count(g, k, nthreads=8) for g in gs] for k in (4, 5)}
    # eager run first: it sizes the workspaces, which the captured run reuses
    o = arb.arb_orient_batch(off, idx, vo, max_graph_n=max_n)
    ws = {k: arb._ws(arb.arb_count_batch_workspace(u.n, u.m, k, len(gs)), "cuda") for k in (4, 5)}
    tots = {k: torch.empty(len(gs), dtype=torch.int64, device="cuda") for k in (4, 5)}
    for k in (4, 5):
        arb.arb_count_batch_async(o["ooff"], o["oidx"], vo, k, totals=tots[k], ws=ws[k])
    torch.cuda.synchronize()
    for k in (4, 5):
        assert [int(x) for x in arb.u64_numpy(tots[k])] == refs[k]
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        cs = torch.cuda.current_stream()
        og = arb.arb_orient_batch(off, idx, vo, max_graph_n=max_n, stream=cs)
        for k in (4, 5):
            arb.arb_count_batch_async(og["ooff"], og["oidx"], vo, k, totals=tots[k], ws=ws[k], stream=cs)
    for rep in range(3):
        for k in (4, 5):
            tots[k].fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        for k in (4, 5):
            assert [int(x) for x in arb.u64_numpy(tots[k])] == refs[k], (k, rep)
