"""The autotuner (arb_autotune) on a mid-size graph: it runs its search, returns options
inside its search space, every candidate gave the same total (else ARB_EMISMATCH), and
counting with the tuned options matches the oracle.  The options cache (tuning.py) stores
the result and returns it without searching again."""
import json
import sys

import pytest
import torch

from paper_2002_10047_amd import graphgen as gg

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def arb():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2002_10047_amd.arb as arb
    return arb


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.mark.parametrize("k", [4, 5])
def test_autotune_search_and_cache(arb, orc, k, tmp_path):
    from paper_2002_10047_amd import tuning
    g = gg.rmat(14, 200000, seed=9)
    off, idx = arb.to_device_csr(g)
    o = arb.arb_orient(off, idx)
    ref = orc.count(g, k, nthreads=8)
    cache = str(tmp_path / "opts.json")
    logs = []
    op, ms = tuning.tuned_opts(o["ooff"], o["oidx"], k, "degree", path=cache, trials=1, log=logs.append)
    say("tuned", k, ms, logs)
    assert ms is not None and ms > 0.0          # the search ran
    d = arb.opts_dict(op)
    space = arb.arb_autotune_space()
    for key, values in space.items():
        assert d[key] in values, (key, d[key], values)
    assert arb.arb_count(o["ooff"], o["oidx"], k, opts=op) == ref
    with open(cache) as f:
        stored = json.load(f)
    assert len(stored) == 1
    op2, ms2 = tuning.tuned_opts(o["ooff"], o["oidx"], k, "degree", path=cache)
    assert ms2 is None and arb.opts_dict(op2) == d        # from the cache, no search
    # learned schedule: the split threshold searched is the cost threshold
    from paper_2002_10047_amd import learn
    w = learn.load_weights(k)
    feat = arb.arb_features(o["ooff"], o["oidx"], o["round"], o["rank"])
    opl, msl = tuning.tuned_opts(o["ooff"], o["oidx"], k, "learned", mlp_weights=w, features=feat, path=cache,
                                 trials=1)
    assert msl > 0.0 and arb.opts_dict(opl)["split_min_cost"] in space["split_min_cost"]
    assert arb.arb_count(o["ooff"], o["oidx"], k, opts=opl) == ref
