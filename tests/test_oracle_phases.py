"""Pins for the oracle's phase tables: one PSF table per depth plane and per position of a point
inside its 2^L x 2^L block (4^L tables per plane), so that points on any pixel, not only on the
2^L grid that the level-scaled shift of Eq.(2) needs, are placed exactly.

* geometry: the table side holds the disk around every shifted centre (hand-worked sides, and a
  brute-force count of the disk's pixels inside the table);
* a phase table is the plane's PSF moved by whole pixels;
* quantisation: nearest pixel, ties upward, table index from the position modulo 2^L (also for
  negative positions), hand-worked;
* with every coefficient kept, WASABI with phase tables equals the circ()-windowed Eq.(1) sum at
  the points' true pixel positions (the paper's one-table-per-plane method does not);
* for one off-grid point and gamma < 1 the squared error is the discarded coefficients' energy.
"""
import numpy as np
import pytest

from workloads import uniform_points

P = 1e-6


def _prm(orc, levels, gamma, phases=1, n_depth=3, dtype=3, max_window=128):
    return orc.LutParams(z_min=20e-6, z_max=70e-6, n_depth=n_depth, levels=levels, gamma=gamma,
                         max_window=max_window, value_dtype=dtype, phases=phases)


def test_phase_geometry_hand_worked(orc):
    # z_d = 20 + (d + 1/2) 50/3 um -> R_d = z_d tan(asin(0.3165)) / 1 um = 9.45, 15.01, 20.57 px
    prm = _prm(orc, 2, 1.0)
    z, R, W, Nr, sx, sy = orc.lut_geometry(prm)
    assert len(z) == 3 * 16
    np.testing.assert_allclose(R[::16], [9.452, 15.013, 20.574], atol=2e-3)
    # W >= 2 floor(R) + 2^(L+1), a multiple of 2^(L+1) = 8: 18 + 8 = 26 -> 32, 30 + 8 = 38 -> 40, 40 + 8 = 48
    assert list(W[::16]) == [32, 40, 48]
    # without phase tables: W >= 2 floor(R) + 2 -> 20 -> 24, 32 -> 32, 42 -> 48
    _, _, W0, _, _, _ = orc.lut_geometry(_prm(orc, 2, 1.0, phases=0))
    assert list(W0) == [24, 32, 48]
    # every table of a plane shares its depth and size; shifts enumerate the 4 x 4 block
    for d in range(3):
        sl = slice(16 * d, 16 * d + 16)
        assert np.all(z[sl] == z[16 * d]) and np.all(W[sl] == W[16 * d]) and np.all(Nr[sl] == W[16 * d] ** 2)
        assert sorted(zip(sy[sl], sx[sl])) == [(a, b) for a in range(4) for b in range(4)]
        assert list(sy[sl] * 4 + sx[sl]) == list(range(16))


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_every_shifted_disk_fits_its_table(orc, levels):
    z, R, W, _, sx, sy = orc.lut_geometry(_prm(orc, levels, 1.0))
    for t in range(0, len(z), max(1, len(z) // 12)):
        T = orc.psf_table(z[t], R[t], int(W[t]), sx=int(sx[t]), sy=int(sy[t]))
        c = np.arange(-60, 61)
        inside = int(np.sum(c[:, None] ** 2 + c[None, :] ** 2 < R[t] ** 2))  # pixels of the disk
        assert int(np.count_nonzero(T)) == inside


def test_phase_table_is_the_moved_psf(orc):
    z, R, W = 50e-6, 12.3, 40
    T0 = orc.psf_table(z, R, W)
    for sx, sy in [(1, 0), (0, 3), (2, 1), (3, 3)]:
        T = orc.psf_table(z, R, W, sx=sx, sy=sy)
        np.testing.assert_array_equal(T[sy:, sx:], T0[:W - sy, :W - sx])
        assert T[W // 2 + sy, W // 2 + sx] == T0[W // 2, W // 2]
        assert abs(T[W // 2 + sy, W // 2 + sx] - np.exp(2j * np.pi * (z / 633e-9 % 1.0))) < 1e-12


def test_phase_quantize_hand_worked(orc):
    prm = _prm(orc, 3, 0.3, n_depth=4)                 # B = 8, 64 phases, dz = 12.5 um
    pts = np.array([[5.4 * P, 9.5 * P, 21e-6, 0.5],     # (5, 10): phase 2*8 + 5, plane 0
                    [-0.6 * P, -8.5 * P, 40e-6, 1.0],   # (-1, -8): phase 0*8 + 7, plane 1
                    [16.0 * P, 7.49 * P, 70e-6, 0.25],  # (16, 7): phase 7*8 + 0, z = z_max -> plane 3
                    [3.0 * P, 3.0 * P, 80e-6, 1.0]])    # beyond z_max: invalid
    q = orc.quantize(pts, prm)
    assert list(q.x) == [5, -1, 16, 0] and list(q.y) == [10, -8, 7, 0]
    assert list(q.d) == [0 * 64 + 21, 1 * 64 + 7, 3 * 64 + 56, -1]
    # the paper's grid: the same points snap to multiples of 8
    q0 = orc.quantize(pts, _prm(orc, 3, 0.3, n_depth=4, phases=0))
    assert list(q0.x[:3]) == [8, 0, 16] and list(q0.y[:3]) == [8, -8, 8] and list(q0.d) == [0, 1, 3, -1]


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_full_phase_lut_equals_direct_sum_off_grid(orc, levels):
    lut = orc.build_lut(_prm(orc, levels, 1.0))
    pts = uniform_points(40 + levels, 30, 150, 120, 20e-6, 70e-6)
    pts[:, 0] -= 40 * P                                 # some points left of / above the window
    pts[:, 1] -= 30 * P
    q = orc.quantize(pts, lut.params)
    B = 1 << levels
    assert np.all(q.d >= 0) and np.any(q.x % B != 0)
    X0, Y0, nx, ny = -2 * B, -B, 12 * B, 10 * B
    u = orc.wasabi(lut, q, X0, Y0, nx, ny)
    ref = orc.direct(orc.snapped_points(q, lut), nx, ny, X0, Y0, window=orc.CIRC)
    assert orc.rel_l2(u, ref) < 1e-12
    # the paper's single table per plane, on the same pixel positions: far off
    lut0 = orc.build_lut(_prm(orc, levels, 1.0, phases=0))
    q0 = orc.Quantized(q.x, q.y, (q.d >> (2 * levels)).astype(np.int32), q.a)
    assert orc.rel_l2(orc.wasabi(lut0, q0, X0, Y0, nx, ny), ref) > 0.1


def test_off_grid_point_error_is_discarded_energy(orc):
    prm = _prm(orc, 3, 0.3)
    lut = orc.build_lut(prm)
    lut_all = orc.build_lut(_prm(orc, 3, 1.0))
    pts = np.array([[61 * P, 66 * P, 60e-6, 0.8]])      # position (5, 2) inside its 8 x 8 block
    q = orc.quantize(pts, prm)
    t = int(q.d[0])
    assert t % 64 == 2 * 8 + 5
    u = orc.wasabi(lut, q, 0, 0, 128, 128)
    ref = orc.wasabi(lut_all, q, 0, 0, 128, 128)
    full = orc.haar_forward(orc.psf_table(lut.z[t], lut.R[t], int(lut.W[t]), sx=5, sy=2), 3).ravel()
    kept = np.zeros(full.size, bool)
    kept[lut.idx[lut.off[t]:lut.off[t + 1]]] = True
    discarded = 0.8 ** 2 * np.sum(np.abs(full[~kept]) ** 2)
    assert abs(np.sum(np.abs(u - ref) ** 2) / discarded - 1) < 1e-10
