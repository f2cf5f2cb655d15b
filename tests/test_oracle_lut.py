"""Pins for the oracle's LUT pre-computation (Sec. 2, step 1): plane geometry, PSF table,
shrinkage selection, storage rounding and point quantisation."""
import numpy as np
import pytest
import torch

from conftest import read_golden

P = 1e-6


def test_plane_geometry_hand_worked(orc):
    (rows,) = read_golden("lut_geometry_2048.txt")
    prm = orc.LutParams(n_depth=64, levels=3, gamma=0.05)
    z, R, W, Nr, _, _ = orc.lut_geometry(prm)
    for d, z_um, R_px, Wd, nr in rows:
        d = int(d)
        assert abs(z[d] * 1e6 - z_um) < 1e-9
        assert abs(R[d] - R_px) < 1e-4
        assert W[d] == Wd and Nr[d] == nr
    assert W.min() == 80 and W.max() == 1008
    assert np.all(W % 16 == 0)
    # gamma >= 1 keeps every coefficient of the table
    _, _, W1, Nr1, _, _ = orc.lut_geometry(orc.LutParams(n_depth=64, levels=3, gamma=1.0))
    np.testing.assert_array_equal(Nr1, W1.astype(np.int64) ** 2)
    with pytest.raises(ValueError):
        orc.lut_geometry(orc.LutParams(n_depth=64, levels=3, max_window=512))


def test_psf_table_closed_forms(orc):
    lam, z = 0.8e-6, 12e-6
    s = lam / (2 * P)
    R = z * (s / np.sqrt(1 - s * s)) / P
    T = orc.psf_table(z, R, 40, P, lam)
    c = 20
    # centre: r = z = 15 wavelengths -> exp(i 2 pi 15) = 1
    assert abs(T[c, c] - 1.0) < 1e-12
    (rows,) = read_golden("direct_pythagorean.txt")
    for dx, dy, re, im, inside in rows:
        expect = complex(re, im) / 0.7 if inside else 0.0
        assert abs(T[c + int(dy), c + int(dx)] - expect) < 1e-12
    # unit modulus inside the disk, zero outside; exact transpose and point symmetry about c
    mag = np.abs(T)
    assert np.all((np.abs(mag - 1) < 1e-14) | (mag == 0))
    np.testing.assert_array_equal(T, T.T)
    np.testing.assert_array_equal(T[1:, 1:], T[1:, 1:][::-1, ::-1])


def test_psf_support_is_gauss_lattice_count(orc):
    T = orc.psf_table(50e-6, 3.2, 16, P, 633e-9)
    assert np.count_nonzero(T) == 37          # sum_{n<=10} r2(n), see the direct-sum pin


def test_selection_is_best_k_by_magnitude(orc):
    rng = np.random.default_rng(3)
    C = rng.normal(size=(16, 16)) + 1j * rng.normal(size=(16, 16))
    C[3, 4] = C[5, 6] = 10.0          # a tie at the top: both kept
    C[0, 1] = C[0, 2] = 0.001j        # a tie at the bottom
    idx, val = orc.select(C, 40)
    assert np.all(np.diff(idx) > 0)
    flat = C.ravel()
    np.testing.assert_array_equal(val, flat[idx])
    kept = np.zeros(256, bool)
    kept[idx] = True
    assert np.abs(flat[kept]).min() >= np.abs(flat[~kept]).max()
    assert {3 * 16 + 4, 5 * 16 + 6} <= set(idx.tolist())
    # tie at the threshold goes to the lower flat index
    D = np.zeros((4, 4), complex)
    D[1, 1] = D[0, 3] = D[2, 0] = 1.0
    idx2, _ = orc.select(D, 2)
    assert idx2.tolist() == [3, 5]
    # strengths equal to single precision count as tied, whichever is larger in FP64
    E = np.zeros((4, 4), complex)
    E[3, 3] = 1.0 + 1e-12
    E[1, 2] = 1.0
    E[0, 0] = 0.5
    idx3, _ = orc.select(E, 1)
    assert idx3.tolist() == [6]


def test_storage_rounding(orc):
    rng = np.random.default_rng(4)
    v = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-9, 6, 2000),
                        [65504.0, 65519.9, 65520.0, 6e-8, 3e-8, 1e-9]])
    for x in v:
        assert orc.round_value(x, orc.F16) == float(np.float16(x)), x
        assert orc.round_value(x, orc.F32) == float(np.float32(x)), x
    # BF16: ties to even, checked by hand and against torch on float32-exact inputs
    assert orc.round_value(1 + 2.0 ** -8, orc.BF16) == 1.0
    assert orc.round_value(1 + 3 * 2.0 ** -8, orc.BF16) == 1 + 2.0 ** -6
    assert orc.round_value(-(1 + 2.0 ** -8 + 2.0 ** -30), orc.BF16) == -(1 + 2.0 ** -7)
    f = rng.normal(size=2000).astype(np.float32) * np.float32(2.0) ** rng.integers(-40, 40, 2000)
    tb = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    for x, t in zip(f.astype(np.float64), tb):
        assert orc.round_value(x, orc.BF16) == t, x


def test_quantize_hand_worked(orc):
    prm = orc.LutParams(n_depth=64, levels=3)
    dz = 1.4e-3 / 64
    pts = np.array([
        [11.9e-6, 0.0, 0.1e-3, 0.5],             # 11.9/8 + 0.5 = 1.9875 -> 8 ; z_min -> plane 0
        [12.0e-6, -4.0e-6, 0.1e-3 + 1.5 * dz, 1.0],  # 12/8 + .5 = 2 -> 16 (ties up); -4 -> 0
        [-4.1e-6, 100e-6, 1.5e-3, 0.25],          # -> -8, 104; z_max -> last plane
        [0.0, 0.0, 0.09e-3, 1.0],                 # below z_min: invalid
        [0.0, 0.0, 1.6e-3, 1.0],                  # above z_max: invalid
        [np.nan, 0.0, 1.0e-3, 1.0],               # not finite: invalid
    ])
    q = orc.quantize(pts, prm)
    assert q.x.tolist() == [8, 16, -8, 0, 0, 0]
    assert q.y.tolist() == [0, 0, 104, 0, 0, 0]
    assert q.d.tolist() == [0, 1, 63, -1, -1, -1]
    np.testing.assert_array_equal(q.a[:3], [0.5, 1.0, 0.25])


@pytest.mark.parametrize("dtype", [0, 1, 2])
def test_lut_entries_are_rounded_top_coefficients(orc, dtype):
    prm = orc.LutParams(z_min=20e-6, z_max=60e-6, n_depth=3, levels=2, gamma=0.3, max_window=64,
                        value_dtype=dtype)
    lut = orc.build_lut(prm)
    for d in range(prm.n_depth):
        W = int(lut.W[d])
        C = orc.haar_forward(orc.psf_table(lut.z[d], lut.R[d], W), prm.levels).ravel()
        sl = slice(lut.off[d], lut.off[d + 1])
        idx, val = lut.idx[sl], lut.val[sl]
        assert len(idx) == lut.Nr[d] and np.all(np.diff(idx) > 0)
        kept = np.zeros(W * W, bool)
        kept[idx] = True
        assert np.abs(C[kept]).min() >= np.abs(C[~kept]).max()
        rounded = np.array([complex(orc.round_value(c.real, dtype), orc.round_value(c.imag, dtype))
                            for c in C[idx]])
        np.testing.assert_array_equal(val, rounded)
