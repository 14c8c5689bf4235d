"""The degree, Goodrich-Pszona and k-core orderings (arb_orient_method) against the
oracle's, byte for byte, and the counts on every ordering against the oracle's."""
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


GRAPHS = [lambda: gg.gnp(400, 0.3, 2), lambda: gg.config_graph("c1"), lambda: gg.rmat(14, 200000, seed=9),
          lambda: gg.rgg(20000, 2, 20.0, 5), lambda: gg.turan(60, 4), lambda: gg.star(50), lambda: gg.empty(3),
          lambda: gg.sbm2(1500, 0.05, 0.8, 7)]


@pytest.mark.parametrize("method", [1, 2, 3])
@pytest.mark.parametrize("gi", range(len(GRAPHS)))
def test_ordering_parity(arb, orc, method, gi):
    g = GRAPHS[gi]()
    eps = 1.0 if method != 2 else 0.5
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient_method(off, idx, method, eps=eps, validate=True)
    r = orc.orient(g, eps, method=method)
    assert np.array_equal(o["round"].cpu().numpy(), r["round"])
    assert np.array_equal(o["deg_at_peel"].cpu().numpy(), r["deg_at_peel"])
    assert np.array_equal(o["rank"].cpu().numpy(), r["rank"])
    assert np.array_equal(o["ooff"].cpu().numpy(), r["ooff"])
    assert np.array_equal(o["oidx"].cpu().numpy(), r["oidx"])
    assert int(o["stats"][0]) == r["rounds"]
    for k in (3, 4, 5):
        assert arb.arb_count(o["ooff"], o["oidx"], k) == orc.count(g, k, nthreads=8), (gi, method, k)
    print(gi, method, "rounds", r["rounds"], file=sys.stderr, flush=True)


def test_ordering_rejects_bad_arguments(arb):
    g = gg.cycle(5)
    off, idx = arb.to_device_csr(g)
    with pytest.raises(Exception):
        arb.arb_orient_method(off, idx, 7)
    with pytest.raises(Exception):
        arb.arb_orient_method(off, idx, arb.ARB_ORIENT_GOODRICH_PSZONA, eps=0.0)
