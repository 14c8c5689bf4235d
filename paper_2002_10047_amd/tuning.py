"""Cache of autotuned counting options, keyed by graph signature, k and schedule.

The search itself is `arb_autotune` in libarb.so; this module only stores and reloads
its results (JSON) so that repeated runs on the same graph skip the search.
"""
from __future__ import annotations

import json
import os

from . import arb

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "count_opts.json")
SCHEDULES = {"degree": arb.ARB_SCHED_PERSISTENT, "learned": arb.ARB_SCHED_LEARNED}


def signature(ooff, oidx) -> str:
    """n, m, largest out-degree and sum of squared out-degrees of a directed CSR."""
    d = (ooff[1:] - ooff[:-1])
    n = ooff.numel() - 1
    return f"n={n},m={oidx.numel()},dmax={int(d.max().item()) if n else 0},d2={int((d * d).sum().item())}"


def _load(path):
    if os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


def tuned_opts(ooff, oidx, k, schedule, mlp_weights=None, features=None, ws=None, retune=False, trials=2,
               path=CACHE, log=None):
    """Options for (graph, k, schedule): from the cache, else from arb_autotune (then cached)."""
    key = f"{signature(ooff, oidx)}|k={k}|{schedule}"
    cache = _load(path)
    op = arb.count_opts(schedule=SCHEDULES[schedule], mlp_weights=mlp_weights, features=features)
    if not retune and key in cache:
        e = cache[key]
        for f in ("split_min_degree", "split_min_cost", "persist_blocks_per_cu", "chunk_small", "bitmap_max_span",
                  "concurrent_tiers", "tier_fill", "big_max_degree"):
            if f in e:
                setattr(op, f, e[f])
        return op, None
    ms = arb.arb_autotune(ooff, oidx, k, op, trials=trials, ws=ws)
    e = arb.opts_dict(op)
    e["ms"] = ms
    cache[key] = e
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    except OSError:
        pass
    if log:
        log(f"tuned {schedule} k={k}: {ms:.3f} ms {e}")
    return op, ms
