"""The counter-based R-MAT and 3-D random geometric graphs built on the GPU (torch) are
byte-identical to the host (numpy) builds from which the oracle's stored totals come."""
import numpy as np
import pytest
import torch

from paper_2002_10047_amd import graphgen as gg

pytestmark = pytest.mark.gpu


def test_rmat_device_equals_host():
    assert torch.cuda.is_available()
    g = gg.rmat_cb_host(16, 16 << 16, seed=51)
    n, off, idx = gg.rmat_cb_device(16, 16 << 16, seed=51, chunk=1 << 18)
    assert n == g.n
    assert np.array_equal(off.cpu().numpy(), g.offsets) and np.array_equal(idx.cpu().numpy(), g.indices)


def test_rgg_device_equals_host():
    g = gg.rgg_cb_host(1 << 17, 40.0, seed=52)
    n, off, idx = gg.rgg_cb_device(1 << 17, 40.0, seed=52, chunk=1 << 15)
    assert np.array_equal(off.cpu().numpy(), g.offsets) and np.array_equal(idx.cpu().numpy(), g.indices)
