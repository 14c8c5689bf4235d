"""The GPU parity cases that target one LDS tier (or the global-scratch kernel) reach it.

Each case below is counted on the GPU in tests/test_gpu_parity.py; its claim about which
tier does the work rests on the out-degrees of the peel orientation (Sec. 3.1, eps = 1).
The GPU orientation is byte-identical to the oracle's (test_orient_parity), so the
oracle's out-degrees decide here, on the CPU, whether each case still reaches its tier."""
import numpy as np
import pytest

import test_gpu_parity as tp
from paper_2002_10047_amd import graphgen as gg


def _outdeg(orc, g):
    r = orc.orient(g, 1.0)
    return np.diff(np.asarray(r["ooff"])), np.asarray(r["rank"])


def test_gnp400_has_128_tier_roots(orc):
    d, _ = _outdeg(orc, gg.gnp(400, 0.3, 2))
    assert ((d > 64) & (d <= 128)).sum() == 196


def test_sbm1500_spans_every_lds_tier(orc):
    d, _ = _outdeg(orc, gg.sbm2(1500, 0.05, 0.8, 7))
    bounds = [(0, 64), (64, 128), (128, 256), (256, 384), (384, 512), (512, 768)]
    assert all(((d > lo) & (d <= hi)).sum() > 0 for lo, hi in bounds)
    assert d.max() <= 768


@pytest.mark.parametrize("name,lo,hi", [
    ("er600_K24", 64, 128), ("er700_K16", 128, 256), ("er1500_K14", 256, 384),
    ("er2000_K13", 384, 512), ("er2600_K12", 512, 768),
])
def test_planted_clique_root_tier(orc, name, lo, hi):
    # every deep clique lies inside the planted clique and is counted from its
    # lowest-ranked member, whose out-degree picks the tier
    mk = {c[0]: c[1] for c in tp.DEEP_K_GRAPHS}[name]
    g = mk()
    d, rank = _outdeg(orc, g)
    first = g.planted[np.argmin(rank[g.planted])]
    assert lo < d[rank[first]] <= hi


def test_sbm2000_k12_root_above_the_lds_tiers(orc):
    g = tp._sbm2000_with_k12()
    d, rank = _outdeg(orc, g)
    base = gg.sbm2(2000, 0.05, 0.85, 11)
    deg = np.diff(np.asarray(base.offsets))
    mem = np.lexsort((np.arange(base.n), deg))[:12]
    first = mem[np.argmin(rank[mem])]
    assert d[rank[first]] > 768
    assert (d > 768).sum() == 279
