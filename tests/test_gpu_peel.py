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


def _k4_iso(z):
    # K_4 plus z isolated vertices: with z = 4, k = 3, eps = 1 every K_4 vertex sits exactly
    # at the removal threshold (Sec. 4.2's "at most")
    u = [a for a in range(4) for b in range(a + 1, 4)]
    v = [b for a in range(4) for b in range(a + 1, 4)]
    return gg.csr_from_pairs(4 + z, np.array(u), np.array(v))


@pytest.mark.parametrize("name,mk", [("c1", lambda: gg.config_graph("c1")), ("gnp", lambda: gg.gnp(600, 0.05, 4)),
                                     ("rmat13", lambda: gg.rmat(13, 100000, seed=4)),
                                     ("K30", lambda: gg.complete(30)), ("empty", lambda: gg.empty(4)),
                                     ("K4+4", lambda: _k4_iso(4)), ("K4+5", lambda: _k4_iso(5))])
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


@pytest.mark.parametrize("name,mk", [("c1", lambda: gg.config_graph("c1")), ("gnp", lambda: gg.gnp(400, 0.06, 4)),
                                     ("rmat11", lambda: gg.rmat(11, 20000, seed=4)),
                                     ("sbm", lambda: gg.sbm2(600, 0.1, 0.3, 3)), ("K20", lambda: gg.complete(20))])
def test_exact_peel_parity(arb, orc, name, mk):
    g = mk()
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx)
    rank = o["rank"].cpu().numpy()
    for k in (3, 4):
        d, r, rnd = arb.arb_peel(o["ooff"], o["oidx"], k)
        dr, rr, rndr = orc.peel(g, k)
        assert (d, r) == (dr, rr), (name, k, d, dr, r, rr)
        assert np.array_equal(rnd.cpu().numpy()[rank], rndr), (name, k)
