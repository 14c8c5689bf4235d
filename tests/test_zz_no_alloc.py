"""arb_count_noalloc (scratch in a file-scope device array, no workspace argument) against
arb_count_async with a caller workspace: totals and per-vertex counts bit-identical, on
two calls in a row, the second with a smaller graph (the array keeps the first call's
contents); a graph whose workspace exceeds the array is rejected before any work."""
import ctypes

import numpy as np
import pytest
import torch

from paper_2002_10047_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def arb():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_10047_amd.arb as arb
    return arb


def reference(arb, o, k):
    n = o["ooff"].numel() - 1
    pv = torch.empty(n, dtype=torch.int64, device="cuda")
    t = arb.arb_count_async(o["ooff"], o["oidx"], k, per_vertex=pv)
    torch.cuda.synchronize()
    return int(arb.u64_numpy(t)[0]), arb.u64_numpy(pv)


def noalloc(arb, o, k, opts=None):
    n = o["ooff"].numel() - 1
    pv = torch.empty(n, dtype=torch.int64, device="cuda")
    t = arb.arb_count_noalloc(o["ooff"], o["oidx"], k, per_vertex=pv, opts=opts)
    torch.cuda.synchronize()
    return int(arb.u64_numpy(t)[0]), arb.u64_numpy(pv)


def test_noalloc_matches_workspace_entry_point(arb):
    big = gg.gnp(1200, 0.2, 5)                 # larger graph first, then a smaller one
    small = gg.gnp(150, 0.5, 1)
    for g, ks in ((big, (3, 4, 5)), (small, (4, 6))):
        off, idx = arb.to_device_csr(g)
        o = arb.arb_orient(off, idx)
        assert arb.arb_count_workspace(g.n, g.m, max(ks)) <= arb.ARB_NOALLOC_SCRATCH_BYTES
        for k in ks:
            t_ref, pv_ref = reference(arb, o, k)
            t, pv = noalloc(arb, o, k)
            assert t == t_ref and np.array_equal(pv, pv_ref), (g.name, k)
            t2, _ = noalloc(arb, o, k, opts=arb.count_opts(schedule=arb.ARB_SCHED_PLAIN))
            assert t2 == t_ref, (g.name, k)


def test_noalloc_rejects_graphs_above_the_limit(arb):
    off = torch.zeros(2, dtype=torch.int64, device="cuda")
    idx = torch.zeros(1, dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    # a descriptor far above the scratch size: rejected before any kernel runs
    dg = arb.ArbOcsr(1 << 30, 1 << 31, off.data_ptr(), idx.data_ptr())
    assert arb.arb_count_workspace(1 << 30, 1 << 31, 4) > arb.ARB_NOALLOC_SCRATCH_BYTES
    rc = arb._lib.arb_count_noalloc(ctypes.byref(dg), 4, ctypes.c_void_p(total.data_ptr()), None, None,
                                    arb._stream())
    assert rc == arb.ARB_ELIMIT
    torch.cuda.synchronize()
