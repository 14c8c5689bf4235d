"""Host replay of the per-vertex counting kernel's LDS index expressions (tests/harness).

Per-vertex counting of the Turan graph T(90,6) at k = 8 once faulted the GPU (memory
aperture violation) in an earlier build.  This CPU test walks every work item of that
case through a model of the current kernel's team LDS (the capacities and row stride of
the two smallest tiers, the member bitmap / hash, the list table of the second level,
the bit rows, the pair ring, the recursion and its per-vertex counters), checking every
index against its array; it also checks the model's counts against the oracle.  All
accesses stay in bounds, so an out-of-range LDS index is not what faulted."""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from paper_2002_10047_amd import graphgen as gg

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "harness", "lds_replay.cpp")


@pytest.fixture(scope="module")
def replay(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("replay") / "liblds_replay.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", so], check=True)
    lib = ctypes.CDLL(so)
    P = ctypes.c_void_p
    lib.lds_replay_count.argtypes = [ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int, P, P]
    lib.lds_replay_count.restype = ctypes.c_uint64

    def run(o, n, k, span_max=1 << 30):
        off = np.ascontiguousarray(o["ooff"], np.int64)
        idx = np.ascontiguousarray(o["oidx"], np.int32)
        if idx.size == 0:
            idx = np.zeros(1, np.int32)
        pv = np.zeros(max(n, 1), np.uint64)
        items = ctypes.c_int64(0)
        t = lib.lds_replay_count(n, off.ctypes.data_as(P), idx.ctypes.data_as(P), k, span_max,
                                 pv.ctypes.data_as(P), ctypes.byref(items))
        return int(t), pv[:n][o["rank"]], items.value      # per-vertex back to original ids
    return run


def test_turan90_k8_in_bounds(replay, orc):
    g = gg.turan(90, 6)
    o = orc.orient(g, 1.0)                  # the GPU's orientation (byte parity is tested)
    for k in range(3, 9):
        t, pv, items = replay(o, g.n, k)
        t_ref, pv_ref = orc.count(g, k, per_vertex=True)
        assert t == t_ref and np.array_equal(pv, pv_ref), k
        assert items > 0
    t, pv, items = replay(o, g.n, 8)
    assert t == 0 and not pv.any()
    assert items == int((np.diff(o["ooff"]) >= 7).sum())      # every root with 7 out-neighbours


@pytest.mark.parametrize("mk,ks", [(lambda: gg.gnp(150, 0.5, 1), (5, 8)), (lambda: gg.complete(40), (6, 8)),
                                   (lambda: gg.turan(70, 7), (6, 8)), (lambda: gg.config_graph("c1"), (4, 8)),
                                   (lambda: gg.gnp(400, 0.3, 2), (7, 8))])
def test_replay_matches_oracle(replay, orc, mk, ks):
    g = mk()
    o = orc.orient(g, 1.0)
    for k in ks:
        for span in (0, 1 << 30):              # hash and id-range bitmap membership
            t, pv, _ = replay(o, g.n, k, span)
            t_ref, pv_ref = orc.count(g, k, per_vertex=True)
            assert t == t_ref and np.array_equal(pv, pv_ref), (g.name, k, span)
    if g.name == "K40":
        assert replay(o, g.n, 8)[0] == math.comb(40, 8)
