"""The benchmark's count of scatter-adds in a window (the algorithmic work of Eq.(2) that its
roofline reports beside the HBM bytes) against the oracle's own superposition: with every stored
value 1 and every amplitude 1, the sum of the oracle's wavelet field over the window is exactly the
number of kept coefficients that land in it.  Points outside the window whose disks reach into it,
several planes and L = 3 and 4 are covered."""
import dataclasses

import numpy as np
import pytest

import bench
from workloads import grid_points


@pytest.mark.parametrize("levels,nx,ny", [(3, 192, 128), (4, 160, 224)])
def test_scatter_add_count_matches_oracle(orc, levels, nx, ny):
    prm = orc.LutParams(z_min=20e-6, z_max=90e-6, n_depth=4, levels=levels, gamma=0.3, max_window=256)
    lut = orc.build_lut(prm)
    ones = dataclasses.replace(lut, val=np.ones_like(lut.val))
    B = 1 << levels
    pts = grid_points(11 + levels, 40, nx + 192, ny + 192, B, 20e-6, 90e-6, x0=-96, y0=-96)
    pts[:, 3] = 1.0
    q = orc.quantize(pts, prm)
    want = orc.superpose(ones, q, 0, 0, nx, ny).real.sum()
    qs = np.stack([q.x, q.y, q.d], axis=1)
    counts = bench.block_counts(lut.off, lut.idx, lut.W, levels)
    got = bench.entries_in_window(qs, counts, lut.W, levels, nx, ny)
    assert got == int(round(want))
    assert got > 1000
