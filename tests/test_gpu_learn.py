"""GPU checks of the scheduling path: features, per-root counts and the instrumented work
measure against the oracle; the MLP forward/backward/Adam kernels against the float64
reference; split parts, learned schedule and batch totals leaving the counts unchanged."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mlp as omlp
from paper_2002_10047_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def arb():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_10047_amd.arb as arb
    return arb


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def orient(arb, g):
    off, idx = arb.to_device_csr(g)
    return arb.arb_orient(off, idx, eps=1.0)


GRAPHS = [lambda: gg.gnp(400, 0.3, 2), lambda: gg.config_graph("c1"), lambda: gg.rmat(13, 100000, seed=4),
          lambda: gg.rgg(6000, 2, 20.0, 3)]


@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_features_per_root_and_work(arb, orc, gi):
    g = GRAPHS[gi]()
    o = orient(arb, g)
    ref = orc.orient(g, 1.0)
    n = g.n
    # features (rank space) against the oracle's definition
    f = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"]).cpu().numpy()
    rr = np.empty(n, np.int64)
    rr[ref["rank"]] = ref["round"]
    fr = orc.features(n, ref["ooff"], ref["oidx"], rr)
    assert np.allclose(f[:, 0], np.log2(1 + fr[:, 0]), rtol=1e-5, atol=1e-5)
    assert np.allclose(f[:, 1], np.log2(1 + fr[:, 1]), rtol=1e-5, atol=1e-5)
    assert np.array_equal(f[:, 2], fr[:, 2])
    # rows of roots below a degree bound are left as they were, the others are the same
    d_all = np.diff(o["ooff"].cpu().numpy())
    for dm in (1, 8, int(arb.ARB_LEARNED_MIN_DEGREE)):
        say("features min_degree", g.name, dm)
        buf = torch.full((3 * n,), float("nan"), dtype=torch.float32, device="cuda")
        fb = arb.arb_features_min_degree(o["ooff"], o["oidx"], o["round"], o["rank"], dm, out=buf).cpu().numpy()
        on = d_all >= dm
        assert np.array_equal(fb[on], f[on])
        assert np.isnan(fb[~on]).all()
    lc = orc.local_cliques(n, ref["ooff"], ref["oidx"], 6)
    d = np.diff(ref["ooff"])
    rows = np.repeat(np.arange(n), d)
    gather = np.bincount(rows, weights=d[ref["oidx"]].astype(np.float64), minlength=n).astype(np.uint64)
    for k in [3, 4, 5, 6]:
        say("work/per-root", g.name, "k", k)
        per_root = torch.empty(n, dtype=torch.int64, device="cuda")
        work = torch.empty(n, dtype=torch.int64, device="cuda")
        tot = arb.arb_count_async(o["ooff"], o["oidx"], k, per_root=per_root)
        arb.arb_count_async(o["ooff"], o["oidx"], k, work=work)
        work2, cyc = arb.arb_count_instrumented(o["ooff"], o["oidx"], k, cycles=True)
        torch.cuda.synchronize()
        assert torch.equal(work2, work)
        live = torch.from_numpy(np.diff(ref["ooff"]) >= k - 1).cuda()
        assert bool((cyc[live] > 0).all()) and bool((cyc[~live] == 0).all())
        torch.cuda.synchronize()
        pr = arb.u64_numpy(per_root)
        assert np.array_equal(pr, lc[:, k - 2])                  # (k-1)-cliques of G[N+(v)]
        assert int(arb.u64_numpy(tot)[0]) == int(lc[:, k - 2].sum())
        wk = arb.u64_numpy(work)
        live = d >= k - 1
        W = ((d + 31) // 32).astype(np.uint64)
        want = gather + W * lc[:, :k - 2].sum(axis=1)
        assert np.array_equal(wk[live], want[live]), k
        assert np.all(wk[~live] == 0)


@pytest.mark.parametrize("split", [1, 3, 16, 100])
def test_split_parts_identical(arb, orc, split):
    g = gg.gnp(400, 0.3, 2)
    o = orient(arb, g)
    for k in [3, 4, 5, 6]:
        t_ref, pv_ref = orc.count(g, k, per_vertex=True, nthreads=8)
        op = arb.count_opts(schedule=arb.ARB_SCHED_PERSISTENT, split_min_degree=split)
        t, pvr = arb.arb_count(o["ooff"], o["oidx"], k, per_vertex=True, opts=op)
        assert t == t_ref
        assert np.array_equal(pvr[o["rank"].cpu().numpy()], pv_ref)


def _rand_params(seed):
    p = omlp.init_params(seed) + np.random.default_rng(seed).normal(0, 0.05, omlp.NPARAM)
    p[omlp.NPARAM - 1] = 0.3
    return p


def test_mlp_forward_backward_against_fp64(arb):
    rng = np.random.default_rng(7)
    p = _rand_params(3)
    bits = omlp.bf16_bits(p)
    pw = omlp.from_bf16_bits(bits).astype(np.float64)          # the weights the GPU sees
    X = (rng.normal(size=(5000, 3)) * np.array([3.0, 5.0, 1.0]) + np.array([4.0, 10.0, 1.0])).astype(np.float32)
    dy = (rng.normal(size=5000) / 5000).astype(np.float32)
    wb = torch.from_numpy(bits.view(np.int16).copy()).cuda()
    Xd = torch.from_numpy(X).cuda()
    y, act = arb.arb_mlp_forward(wb, Xd, want_act=True)
    y_ref, cache = omlp.forward(pw, X.astype(np.float64))
    y = y.cpu().numpy()
    assert np.max(np.abs(y - y_ref)) <= 1e-4 * max(1.0, np.max(np.abs(y_ref)))
    # inference without activations runs on the matrix cores (activations as bf16 hi + lo)
    for rows in (5000, 16, 1, 33):
        yi = arb.arb_mlp_forward(wb, Xd[:rows].contiguous()).cpu().numpy()
        assert yi.shape == (rows,)
        assert np.max(np.abs(yi - y_ref[:rows])) <= 1e-4 * max(1.0, np.max(np.abs(y_ref))), rows
    act = act.cpu().numpy().reshape(-1, 192)
    assert np.allclose(act[:, :64], cache[1], atol=1e-4 * max(1.0, np.abs(cache[1]).max()))
    g = arb.arb_mlp_backward(wb, Xd, torch.from_numpy(act.ravel().copy()).cuda(), torch.from_numpy(dy).cuda())
    g = g.cpu().numpy()
    g_ref = omlp.backward(pw, cache, dy.astype(np.float64))
    assert np.max(np.abs(g - g_ref)) <= 1e-3 * np.max(np.abs(g_ref))


def test_mse_and_adam_against_fp64(arb):
    rng = np.random.default_rng(1)
    y = rng.normal(size=777).astype(np.float32)
    t = rng.normal(size=777).astype(np.float32)
    dy, loss = arb.arb_mse_grad(torch.from_numpy(y).cuda(), torch.from_numpy(t).cuda())
    L, dy_ref = omlp.loss_and_dy(y, t)
    assert abs(float(loss.item()) - L) <= 1e-5 * abs(L)
    assert np.allclose(dy.cpu().numpy(), dy_ref, rtol=1e-5, atol=1e-9)
    w = rng.normal(size=omlp.NPARAM).astype(np.float32)
    gr = rng.normal(size=omlp.NPARAM).astype(np.float32)
    m = (rng.normal(size=omlp.NPARAM) * 0.01).astype(np.float32)
    v = (rng.random(omlp.NPARAM) * 0.01).astype(np.float32)
    wd, md, vd = (torch.from_numpy(a.copy()).cuda() for a in (w, m, v))
    wb = torch.empty(omlp.NPARAM, dtype=torch.int16, device="cuda")
    arb.arb_adam_step(wd, wb, torch.from_numpy(gr).cuda(), md, vd, 1e-3, 5)
    w_ref, m_ref, v_ref = omlp.adam_step(w.astype(np.float64), gr.astype(np.float64), m.astype(np.float64),
                                         v.astype(np.float64), 1e-3, 5)
    assert np.allclose(wd.cpu().numpy(), w_ref, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), m_ref, rtol=1e-5, atol=1e-7)
    assert np.allclose(vd.cpu().numpy(), v_ref, rtol=1e-4, atol=1e-9)
    assert np.array_equal(wb.cpu().numpy().view(np.uint16), omlp.bf16_bits(wd.cpu().numpy()))


def test_training_reduces_loss_and_learned_counts_identical(arb, orc):
    from paper_2002_10047_amd import learn
    gs = gg.batch_mix(18, m_lo=3e3, m_hi=3e4, seed_base=500)
    k = 4
    rows = [learn.graph_rows(g, k) for g in gs]
    Xtr = torch.cat([r[0] for r in rows[:12]])
    ytr = torch.cat([r[1] for r in rows[:12]])
    Xva = torch.cat([r[0] for r in rows[12:]])
    yva = torch.cat([r[1] for r in rows[12:]])
    tr, hist = learn.train(Xtr, ytr, steps=600, batch=2048, lr=3e-3, Xval=Xva, yval=yva, log_every=200, log=say)
    v0 = learn.Trainer(seed=0).loss(Xva, yva)
    assert hist[-1][2] < 0.25 * v0, (v0, hist)
    g = gg.gnp(400, 0.3, 2)
    o = orient(arb, g)
    feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])
    for kk in [3, 4, 5]:
        t_ref, pv_ref = orc.count(g, kk, per_vertex=True, nthreads=8)
        for sc in [0.0, 4.0, 12.0]:
            op = arb.count_opts(schedule=arb.ARB_SCHED_LEARNED, split_min_cost=sc, mlp_weights=tr.wb, features=feat)
            t, pvr = arb.arb_count(o["ooff"], o["oidx"], kk, per_vertex=True, opts=op)
            assert t == t_ref
            assert np.array_equal(pvr[o["rank"].cpu().numpy()], pv_ref)


def test_batch_totals_and_graph_replay(arb, orc):
    gs = gg.batch_mix(12, m_lo=2e3, m_hi=2e4, seed_base=900)
    u, vo = gg.disjoint_union(gs)
    off, idx = arb.to_device_csr(u)
    o = arb.arb_orient(off, idx, eps=1.0)
    vod = torch.from_numpy(vo).cuda()
    refs = {k: [orc.count(g, k) for g in gs] for k in (4, 5)}
    n = u.n
    for k in (4, 5):
        ws = arb.CountWorkspace(o["ooff"], o["oidx"], k)
        per_root = torch.empty(n, dtype=torch.int64, device="cuda")
        total = torch.empty(1, dtype=torch.int64, device="cuda")
        arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, ws=ws)   # eager warm-up
        torch.cuda.synchronize()
        eager = [int(x) for x in arb.u64_numpy(arb.arb_segment_sum_u64(arb.arb_permute_u64(o["rank"], per_root), vod))]
        assert eager == refs[k]
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=s):
            arb.arb_count_async(o["ooff"], o["oidx"], k, total=total, per_root=per_root, ws=ws,
                                stream=torch.cuda.current_stream())
            per_orig = arb.arb_permute_u64(o["rank"], per_root, stream=torch.cuda.current_stream())
            totals = arb.arb_segment_sum_u64(per_orig, vod, stream=torch.cuda.current_stream())
        for rep in range(3):
            total.fill_(0)
            per_root.fill_(7)
            torch.cuda.synchronize()
            graph.replay()
            torch.cuda.synchronize()
            got = [int(x) for x in arb.u64_numpy(totals)]
            assert got == refs[k], (k, rep)
            assert int(arb.u64_numpy(total)[0]) == sum(refs[k])
