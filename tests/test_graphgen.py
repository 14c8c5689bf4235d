"""The counter-based generators: SplitMix64 against its published outputs, and the torch
build of the R-MAT and 3-D random geometric graphs byte-identical to the numpy build (on
the CPU here; tests/test_gpu_generators.py repeats it on the GPU)."""
import numpy as np
import torch

from paper_2002_10047_amd import graphgen as gg


def test_splitmix64_reference_outputs():
    # the first outputs of SplitMix64 seeded with 1234567, as printed by its authors'
    # reference implementation
    ref = [6457827717110365317, 3203168211198807973, 9817491932198370423, 4593380528125082431,
           16408922859458223821]
    assert [int(x) for x in gg.sm64_np(1234567, np.arange(5))] == ref
    t = gg.sm64_torch(1234567, torch.arange(5, dtype=torch.int64))
    assert [int(x) % (1 << 64) for x in t.tolist()] == ref
    # draw i is a function of i alone: any subset of indices gives the same values
    idx = np.array([7, 1 << 40, 3, (1 << 62) + 5])
    full = gg.sm64_np(99, idx)
    assert [int(gg.sm64_np(99, np.array([i]))[0]) for i in idx] == [int(x) for x in full]


def test_uniform_draws():
    u = gg.unif_np(gg.stream_key(5, 1), np.arange(1 << 16))
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01
    ut = gg.unif_torch(gg.stream_key(5, 1), torch.arange(1 << 16, dtype=torch.int64)).numpy()
    assert np.array_equal(u, ut)


def test_rmat_torch_equals_numpy(orc):
    for scale, seed in ((9, 3), (11, 51)):
        g = gg.rmat_cb_host(scale, 16 << scale, seed=seed, chunk=1 << 12)
        n, off, idx = gg.rmat_cb_device(scale, 16 << scale, seed=seed, device="cpu", chunk=1 << 13)
        assert n == g.n and np.array_equal(off.numpy(), g.offsets) and np.array_equal(idx.numpy(), g.indices)
        assert orc.validate(g) == 0
        assert g.m > 0.8 * (16 << scale) / 2


def test_rgg_torch_equals_numpy(orc):
    for n, deg, seed in ((3000, 20.0, 1), (10000, 40.0, 52)):
        g = gg.rgg_cb_host(n, deg, seed=seed)
        n2, off, idx = gg.rgg_cb_device(n, deg, seed=seed, device="cpu")
        assert np.array_equal(off.numpy(), g.offsets) and np.array_equal(idx.numpy(), g.indices)
        assert orc.validate(g) == 0
        assert abs(2 * g.m / n - deg) < 0.05 * deg
