"""arb-approx-peel on the GPU (Sec. 4.2) against the oracle's: the same rounds, best
density and best vertex set (mapped from rank space)."""
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


@pytest.mark.parametrize("name,mk", [("c1", lambda: gg.config_graph("c1")), ("gnp", lambda: gg.gnp(600, 0.05, 4)),
                                     ("rmat13", lambda: gg.rmat(13, 100000, seed=4)),
                                     ("K30", lambda: gg.complete(30)), ("empty", lambda: gg.empty(4))])
def test_approx_peel_parity(arb, orc, name, mk):
    g = mk()
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx)
    rank = o["rank"].cpu().numpy()
    for k, eps in ((2, 0.5), (3, 1.0), (4, 0.25), (5, 0.5)):
        d, r, mask = arb.arb_approx_peel(o["ooff"], o["oidx"], k, eps)
        dr, rr, mr = orc.approx_peel(g, k, eps)
        assert (d, r) == (dr, rr), (name, k, eps)
        assert np.array_equal(mask.cpu().numpy()[rank] != 0, mr), (name, k, eps)
