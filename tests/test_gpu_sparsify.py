"""Colorful sparsification on the GPU (Sec. 3.3): the sparsified CSR is byte-identical
to the oracle's for the same colours, its k-clique counts equal the oracle's, and the
estimate is count * c^(k-1)."""
import sys

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


@pytest.mark.parametrize("name,mk", [("gnp", lambda: gg.gnp(3000, 0.01, 3)), ("c1", lambda: gg.config_graph("c1")),
                                     ("rmat14", lambda: gg.rmat(14, 200000, seed=9)),
                                     ("sbm1500", lambda: gg.sbm2(1500, 0.05, 0.8, 7))])
def test_sparsify_and_count(arb, orc, name, mk):
    g = mk()
    off, idx = arb.to_device_csr(g)
    for c, seed in ((1, 1), (2, 2), (4, 3), (16, 4)):
        col = gg.colors(g.n, c, seed)
        h = orc.sparsify(g, col)
        soff, sidx = arb.arb_sparsify(off, idx, torch.from_numpy(col).cuda())
        assert np.array_equal(soff.cpu().numpy(), h.offsets)
        assert np.array_equal(sidx.cpu().numpy(), h.indices)
        o = arb.arb_orient(soff, sidx, validate=True)
        for k in (3, 4, 5):
            want = orc.count(h, k, nthreads=8)
            got = arb.arb_count(o["ooff"], o["oidx"], k)
            assert got == want, (name, c, k)
            assert arb.arb_colorful_estimate(got, c, k) == orc.colorful_estimate(want, c, k)
    print(name, "ok", file=sys.stderr, flush=True)


def test_sparsify_edge_cases(arb):
    g = gg.empty(1)
    off, idx = arb.to_device_csr(g)
    soff, sidx = arb.arb_sparsify(off, idx, torch.zeros(1, dtype=torch.int32, device="cuda"))
    assert soff.cpu().tolist() == [0, 0] and sidx.numel() == 0
    with pytest.raises(Exception):
        arb.arb_colorful_estimate(5, 0, 3)
