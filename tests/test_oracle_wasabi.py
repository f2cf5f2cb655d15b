"""Pins for the oracle's wavelet-domain superposition, Eq.(2), with the sub-hologram shift of the
large-scale procedure (Sec. 2) and the inverse transform.

* with every coefficient kept (gamma >= 1) and points on the 2^L grid, WASABI equals the
  circ()-windowed Eq.(1) sum exactly (up to rounding);
* for gamma < 1 it equals the spatial superposition of the shrunk PSFs, placed by brute force;
* for one point the squared error equals the energy of the discarded coefficients (Parseval);
* sub-hologram tiling, shifts on the 2^L grid and amplitude scaling behave as the method says.
"""
import numpy as np
import pytest

from workloads import grid_points

P = 1e-6


def _small_lut(orc, levels, gamma, dtype=3, n_depth=4):
    prm = orc.LutParams(z_min=20e-6, z_max=70e-6, n_depth=n_depth, levels=levels, gamma=gamma,
                        max_window=128, value_dtype=dtype)
    return orc.build_lut(prm)


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_full_lut_equals_windowed_direct_sum(orc, levels):
    lut = _small_lut(orc, levels, gamma=1.0)
    B = 1 << levels
    # points on the grid, some outside the window; window origin negative and not square
    pts = grid_points(10 + levels, 40, 160, 128, B, 20e-6, 70e-6, x0=-32, y0=-48)
    q = orc.quantize(pts, lut.params)
    assert np.all(q.d >= 0)
    X0, Y0, nx, ny = -16, -32, 96, 64
    u = orc.wasabi(lut, q, X0, Y0, nx, ny)
    ref = orc.direct(orc.snapped_points(q, lut), nx, ny, X0, Y0, window=orc.CIRC)
    assert orc.rel_l2(u, ref) < 1e-12


def _dense_kept(orc, lut, d):
    W = int(lut.W[d])
    S = np.zeros(W * W, complex)
    sl = slice(lut.off[d], lut.off[d + 1])
    S[lut.idx[sl]] = lut.val[sl]
    return S.reshape(W, W)


@pytest.mark.parametrize("levels,gamma", [(2, 0.2), (3, 0.05), (3, 0.6), (4, 0.3)])
def test_shrunk_superposition_equals_spatial_placement(orc, levels, gamma):
    lut = _small_lut(orc, levels, gamma)
    B = 1 << levels
    pts = grid_points(20 + levels, 30, 192, 160, B, 20e-6, 70e-6, x0=-48, y0=-16)
    q = orc.quantize(pts, lut.params)
    X0, Y0, nx, ny = -32, 0, 128, 96
    u = orc.wasabi(lut, q, X0, Y0, nx, ny)
    # brute force: shrunk PSF of each plane back in space, added at the point's table origin
    ref = np.zeros((ny, nx), complex)
    kernels = {d: orc.haar_inverse(_dense_kept(orc, lut, d), levels) for d in set(q.d.tolist())}
    for j in range(len(q.d)):
        K = kernels[int(q.d[j])]
        W = K.shape[0]
        r0, c0 = int(q.y[j]) - W // 2 - Y0, int(q.x[j]) - W // 2 - X0
        for r in range(W):
            rr = r0 + r
            if 0 <= rr < ny:
                lo, hi = max(0, -c0), min(W, nx - c0)
                if lo < hi:
                    ref[rr, c0 + lo:c0 + hi] += q.a[j] * K[r, lo:hi]
    assert orc.rel_l2(u, ref) < 1e-12


def test_single_point_error_is_discarded_energy(orc):
    lut_all = _small_lut(orc, 3, gamma=1.0)
    lut = _small_lut(orc, 3, gamma=0.3)
    pts = np.array([[64 * P, 64 * P, 60e-6, 0.8]])
    q = orc.quantize(pts, lut.params)
    d = int(q.d[0])
    u = orc.wasabi(lut, q, 0, 0, 128, 128)
    ref = orc.wasabi(lut_all, q, 0, 0, 128, 128)
    full = orc.haar_forward(orc.psf_table(lut.z[d], lut.R[d], int(lut.W[d])), 3).ravel()
    kept = np.zeros(full.size, bool)
    kept[lut.idx[lut.off[d]:lut.off[d + 1]]] = True
    discarded = 0.8 ** 2 * np.sum(np.abs(full[~kept]) ** 2)
    err = np.sum(np.abs(u - ref) ** 2)
    assert abs(err / discarded - 1) < 1e-10


def test_tiling_shift_and_linearity(orc):
    lut = _small_lut(orc, 3, gamma=0.25)
    pts = grid_points(7, 25, 128, 128, 8, 20e-6, 70e-6)
    q = orc.quantize(pts, lut.params)
    whole = orc.wasabi(lut, q, 0, 0, 128, 128)
    # sub-holograms (s, t) of 64 x 64 reassemble the whole hologram (Sec. 2 large-scale steps 2-4)
    for t in range(2):
        for s in range(2):
            sub = orc.wasabi(lut, q, 64 * s, 64 * t, 64, 64)
            np.testing.assert_allclose(sub, whole[64 * t:64 * t + 64, 64 * s:64 * s + 64], atol=1e-13)
    # moving every point and the window by the same multiple of 2^L changes nothing
    q2 = orc.Quantized(q.x + 40, q.y - 24, q.d, q.a)
    np.testing.assert_allclose(orc.wasabi(lut, q2, 40, -24, 128, 128), whole, atol=1e-13)
    # linear in the amplitudes
    q3 = orc.Quantized(q.x, q.y, q.d, 2.5 * q.a)
    np.testing.assert_allclose(orc.wasabi(lut, q3, 0, 0, 128, 128), 2.5 * whole, atol=1e-12)
    # invalid points contribute nothing
    q4 = orc.Quantized(q.x, q.y, np.where(np.arange(25) % 2 == 0, q.d, -1).astype(np.int32), q.a)
    keep = np.arange(25) % 2 == 0
    q5 = orc.Quantized(q.x[keep], q.y[keep], q.d[keep], q.a[keep])
    np.testing.assert_array_equal(orc.wasabi(lut, q4, 0, 0, 128, 128),
                                  orc.wasabi(lut, q5, 0, 0, 128, 128))


def test_off_grid_positions_floor_to_the_grid(orc):
    # positions that are not multiples of 2^L are floored to the grid (also below zero)
    lut = _small_lut(orc, 3, gamma=0.25)
    x = np.array([-3, 13, 40], np.int32); y = np.array([21, -9, -1], np.int32)
    d = np.array([0, 1, 3], np.int32); a = np.array([0.5, 1.0, 0.75])
    off_grid = orc.wasabi(lut, orc.Quantized(x, y, d, a), -32, -32, 96, 96)
    floored = orc.Quantized(np.array([-8, 8, 40], np.int32), np.array([16, -16, -8], np.int32), d, a)
    np.testing.assert_array_equal(off_grid, orc.wasabi(lut, floored, -32, -32, 96, 96))
    moved = orc.Quantized(np.array([0, 16, 48], np.int32), np.array([24, -8, 0], np.int32), d, a)
    assert np.abs(orc.wasabi(lut, moved, -32, -32, 96, 96) - off_grid).max() > 1e-3
