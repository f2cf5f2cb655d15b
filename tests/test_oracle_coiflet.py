"""Pins for the oracle's coiflet path (the wavelet the paper names, Sec. 2; order 1, six taps).

* filter bank: orthonormal (unit energy, orthogonal to its even shifts, sum sqrt 2); the wavelet
  filter has vanishing moments of order 0 and 1 and the scaling filter vanishing moments of
  order 1 and 2 about its centre -- the properties that define a coiflet, not re-typed values;
* the periodised 2-D transform: perfect reconstruction, Parseval, Haar's filters reproduce the
  Haar transform, a ramp has no interior level-1 details;
* WASABI with a full coiflet LUT (gamma >= 1) equals the circ()-windowed Eq.(1) sum exactly on the
  window (the halo keeps the filters' reach and the periodic wrap outside it), for several L;
* one point: the squared error equals the energy of the discarded coefficients;
* sub-holograms, each with its own halo, reassemble the whole hologram.
"""
import numpy as np
import pytest

from workloads import grid_points

P = 1e-6


def test_coiflet_filter_bank(orc):
    lo, hi = orc.filters(orc.COIF1)
    assert len(lo) == 6
    assert abs(lo.sum() - np.sqrt(2)) < 1e-14 and abs(np.dot(lo, lo) - 1) < 1e-14
    for m in (1, 2):                                 # orthogonal to its shifts by 2 and 4
        assert abs(np.dot(lo[2 * m:], lo[:6 - 2 * m])) < 1e-14
    n = np.arange(6)
    assert abs(hi.sum()) < 1e-14 and abs(np.dot(n, hi)) < 1e-13          # wavelet moments 0, 1
    centre = np.dot(n, lo) / lo.sum()
    assert abs(centre - 2) < 1e-13                                        # integer centre
    assert abs(np.dot((n - centre) ** 2, lo)) < 1e-13                     # scaling moment 2
    assert abs(np.dot(lo, hi)) < 1e-14 and abs(np.dot(hi, hi) - 1) < 1e-14
    hlo, hhi = orc.filters(orc.HAAR)
    np.testing.assert_allclose(hlo, [2 ** -0.5] * 2)
    np.testing.assert_allclose(hhi, [2 ** -0.5, -(2 ** -0.5)])


@pytest.mark.parametrize("wavelet,levels,shape", [(1, 1, (16, 24)), (1, 3, (64, 48)), (1, 4, (96, 128)),
                                                  (0, 3, (32, 40))])
def test_transform_reconstructs_and_keeps_energy(orc, wavelet, levels, shape):
    rng = np.random.default_rng(levels)
    a = rng.normal(size=shape) + 1j * rng.normal(size=shape)
    C = orc.dwt_forward(a, levels, wavelet)
    np.testing.assert_allclose(orc.dwt_inverse(C, levels, wavelet), a, atol=1e-12)
    assert abs(np.linalg.norm(C) / np.linalg.norm(a) - 1) < 1e-13


def test_haar_filters_give_the_haar_transform(orc):
    rng = np.random.default_rng(9)
    a = rng.normal(size=(32, 64)) + 1j * rng.normal(size=(32, 64))
    np.testing.assert_allclose(orc.dwt_forward(a, 3, orc.HAAR), orc.haar_forward(a, 3), atol=1e-13)


def test_ramp_has_no_interior_details(orc):
    x = np.tile(np.arange(64, dtype=float), (8, 1)) + 0j       # linear along x, constant along y
    C = orc.dwt_forward(x, 1, orc.COIF1)
    details_x = C[:4, 32:]                                      # H band: detail along x
    assert np.abs(details_x[:, :30]).max() < 1e-11              # away from the periodic wrap
    assert np.abs(details_x[:, 30:]).max() > 1.0                # the wrap itself is not smooth
    assert np.abs(C[4:, :]).max() < 1e-11                       # constant along y: no V, D


def _lut(orc, levels, gamma, n_depth=3, dtype=3):
    return orc.build_lut(orc.LutParams(z_min=20e-6, z_max=70e-6, n_depth=n_depth, levels=levels, gamma=gamma,
                                       max_window=512, value_dtype=dtype, wavelet=orc.COIF1))


@pytest.mark.parametrize("levels", [1, 2, 3])
def test_full_coiflet_lut_equals_windowed_direct_sum(orc, levels):
    lut = _lut(orc, levels, 1.0)
    B = 1 << levels
    pts = grid_points(50 + levels, 25, 160, 128, B, 20e-6, 70e-6, x0=-32, y0=-48)
    q = orc.quantize(pts, lut.params)
    X0, Y0, nx, ny = -2 * B, -B, 12 * B, 10 * B
    u = orc.wasabi(lut, q, X0, Y0, nx, ny)
    ref = orc.direct(orc.snapped_points(q, lut), nx, ny, X0, Y0, window=orc.CIRC)
    assert orc.rel_l2(u, ref) < 1e-12
    # without the halo the filters' reach and the periodic wrap spoil the window
    bare = orc.dwt_inverse(orc.superpose(lut, q, X0, Y0, nx, ny), levels, orc.COIF1)
    assert orc.rel_l2(bare, ref) > 1e-3


def test_coiflet_single_point_error_is_discarded_energy(orc):
    lut_all, lut = _lut(orc, 3, 1.0), _lut(orc, 3, 0.3)
    pts = np.array([[64 * P, 56 * P, 60e-6, 0.8]])
    q = orc.quantize(pts, lut.params)
    d = int(q.d[0])
    u = orc.wasabi(lut, q, 0, 0, 128, 128)
    ref = orc.wasabi(lut_all, q, 0, 0, 128, 128)
    full = orc.dwt_forward(orc.psf_table(lut.z[d], lut.R[d], int(lut.W[d])), 3, orc.COIF1).ravel()
    kept = np.zeros(full.size, bool)
    kept[lut.idx[lut.off[d]:lut.off[d + 1]]] = True
    discarded = 0.8 ** 2 * np.sum(np.abs(full[~kept]) ** 2)
    assert abs(np.sum(np.abs(u - ref) ** 2) / discarded - 1) < 1e-9


def test_coiflet_sub_holograms_reassemble(orc):
    lut = _lut(orc, 3, 0.25)
    pts = grid_points(7, 25, 128, 128, 8, 20e-6, 70e-6)
    q = orc.quantize(pts, lut.params)
    whole = orc.wasabi(lut, q, 0, 0, 128, 128)
    for t in range(2):
        for s in range(2):
            sub = orc.wasabi(lut, q, 64 * s, 64 * t, 64, 64)
            np.testing.assert_allclose(sub, whole[64 * t:64 * t + 64, 64 * s:64 * s + 64], atol=1e-12)
