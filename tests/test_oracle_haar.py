"""Pins for the oracle's Haar transform (Sec. 2 steps 1 and 3, Fig. 2(a) layout).

The oracle builds the transform from the recursive 2x2 rule.  These tests check it against
(a) a hand-worked fixture, (b) an independent construction from the Haar basis functions,
(c) perfect reconstruction and energy conservation, (d) the constant-block closed form.
"""
import numpy as np
import pytest

from conftest import read_golden


def test_hand_worked_2x2(orc):
    a = np.array([[1.0, 2.0], [3.0, 4.0]])
    # S=(1+2+3+4)/2=5, H=(1-2+3-4)/2=-1, V=(1+2-3-4)/2=-2, D=(1-2-3+4)/2=0
    np.testing.assert_array_equal(orc.haar_forward(a, 1).real, [[5.0, -1.0], [-2.0, 0.0]])


def test_hand_worked_4x4(orc):
    src, lev1, lev2 = read_golden("haar_4x4.txt")
    np.testing.assert_array_equal(orc.haar_forward(src, 1).real, lev1)
    np.testing.assert_array_equal(orc.haar_forward(src, 2).real, lev2)
    np.testing.assert_array_equal(orc.haar_inverse(lev2, 2).real, src)


def _phi(level, size):
    """Rows: scaling functions of width 2^level, value 2^(-level/2) on their support."""
    w = 1 << level
    m = np.zeros((size // w, size))
    for k in range(size // w):
        m[k, k * w:(k + 1) * w] = 2.0 ** (-level / 2)
    return m


def _psi(level, size):
    """Rows: Haar wavelets of width 2^level, +2^(-level/2) on the first half, - on the second."""
    w = 1 << level
    m = np.zeros((size // w, size))
    for k in range(size // w):
        m[k, k * w:k * w + w // 2] = 2.0 ** (-level / 2)
        m[k, k * w + w // 2:(k + 1) * w] = -(2.0 ** (-level / 2))
    return m


def _haar_by_basis(a, levels):
    """Mallat-layout coefficients as inner products with the 2D (non-standard) Haar basis."""
    h, w = a.shape
    out = np.zeros_like(a)
    for l in range(1, levels + 1):
        pr, sr = _phi(l, h), _psi(l, h)
        pc, sc = _phi(l, w), _psi(l, w)
        bh, bw = h >> l, w >> l
        out[0:bh, bw:2 * bw] = pr @ a @ sc.T        # H: wavelet along columns (x)
        out[bh:2 * bh, 0:bw] = sr @ a @ pc.T        # V: wavelet along rows (y)
        out[bh:2 * bh, bw:2 * bw] = sr @ a @ sc.T   # D: wavelet along both
    bh, bw = h >> levels, w >> levels
    out[0:bh, 0:bw] = _phi(levels, h) @ a @ _phi(levels, w).T
    return out


@pytest.mark.parametrize("levels,h,w", [(1, 4, 6), (2, 8, 8), (3, 16, 24), (4, 32, 16)])
def test_matches_basis_functions(orc, levels, h, w):
    rng = np.random.default_rng(levels)
    a = rng.normal(size=(h, w)) + 1j * rng.normal(size=(h, w))
    ref = _haar_by_basis(a.real, levels) + 1j * _haar_by_basis(a.imag, levels)
    np.testing.assert_allclose(orc.haar_forward(a, levels), ref, rtol=0, atol=1e-12)


@pytest.mark.parametrize("levels,h,w", [(1, 2, 2), (3, 24, 40), (4, 64, 32), (5, 64, 64)])
def test_perfect_reconstruction_and_energy(orc, levels, h, w):
    rng = np.random.default_rng(100 + levels)
    a = rng.normal(size=(h, w)) + 1j * rng.normal(size=(h, w))
    c = orc.haar_forward(a, levels)
    assert abs(np.sum(np.abs(c) ** 2) / np.sum(np.abs(a) ** 2) - 1) < 1e-13
    np.testing.assert_allclose(orc.haar_inverse(c, levels), a, rtol=0, atol=1e-13)


@pytest.mark.parametrize("levels", [1, 2, 3, 4])
def test_constant_block_gives_one_coefficient(orc, levels):
    b = 1 << levels
    c = orc.haar_forward(np.full((b, b), 0.75 - 0.25j), levels)
    expect = np.zeros((b, b), complex)
    expect[0, 0] = (2 ** levels) * (0.75 - 0.25j)
    np.testing.assert_allclose(c, expect, atol=1e-15)
