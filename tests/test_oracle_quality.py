"""Pins of the oracle's quality measures: PSNR and relative L2 error.

The paper judges holograms by their look and prints no quality figure, so these measures are
readings, not passages: PSNR = 10 log10(max|u_ref|^2 / mean|u - u_ref|^2) on the complex field
(the peak power of the reference over the mean power of the error), rel-L2 = ||u - u_ref|| / ||u_ref||.
The 40 dB selectivity of the benchmarks comes out of `psnr` (through the selectivity sweep), and
several pins assert `rel_l2(...) < tol`, so both are pinned here on hand-worked values, and each
plausible mistake (peak taken from the wrong field, magnitude for power, the wrong norm in the
denominator) is planted and shown to fail these pins.
"""
import math

import numpy as np
import pytest


def check_psnr(psnr):
    """Hand-worked values.  Reference peak |2| (power 4); the error is 0.1 in magnitude at every
    element (mean power 0.01), so PSNR = 10 log10(4 / 0.01) = 26.0206 dB.  The approximation's own
    peak is 2.1, so a PSNR that took the peak from it would give 10 log10(4.41 / 0.01)."""
    ref = np.array([2.0, 1j, -1.0, 0.5 + 0.5j])
    err = np.array([0.1, 0.1j, -0.1, 0.1 * np.exp(0.3j)])
    u = ref + err
    assert psnr(u, ref) == pytest.approx(10 * math.log10(4 / 0.01), abs=1e-9)
    assert psnr(u, ref) == pytest.approx(26.020599913279625, abs=1e-9)
    # the arguments are not interchangeable: the peak is the reference's
    assert psnr(ref, u) == pytest.approx(10 * math.log10(2.1 ** 2 / 0.01), abs=1e-9)
    # a 2-D field: one element off by 3 in 9, peak 5 -> 10 log10(25 / (9 / 9)) = 13.979 dB
    r2 = np.zeros((3, 3), complex)
    r2[1, 2] = 5j
    u2 = r2.copy()
    u2[0, 0] = 3.0
    assert psnr(u2, r2) == pytest.approx(10 * math.log10(25.0), abs=1e-9)
    # exact -> infinite
    assert psnr(ref.copy(), ref) == math.inf


def check_rel_l2(rel_l2):
    """||(3, 4i + 1) - (3, 4i)|| / ||(3, 4i)|| = 1 / 5 exactly; with ||u|| in the denominator it
    would be 1 / sqrt(26)."""
    ref = np.array([3.0, 4j])
    u = np.array([3.0, 4j + 1.0])
    assert rel_l2(u, ref) == pytest.approx(0.2, abs=1e-15)
    assert rel_l2(ref, u) == pytest.approx(1.0 / math.sqrt(26.0), abs=1e-15)
    # norms over all elements of a 2-D array, not per row
    r2 = np.array([[3.0, 0.0], [0.0, 4.0]])
    u2 = r2 + np.array([[0.0, 0.0], [0.0, 0.5]])
    assert rel_l2(u2, r2) == pytest.approx(0.1, abs=1e-15)
    assert rel_l2(ref, ref) == 0.0


def test_psnr_pinned(orc):
    check_psnr(orc.psnr)


def test_rel_l2_pinned(orc):
    check_rel_l2(orc.rel_l2)


def _psnr_peak_from_u(u, ref):
    mse = float(np.mean(np.abs(u - ref) ** 2))
    return 10 * math.log10(float(np.max(np.abs(u)) ** 2) / mse)


def _psnr_magnitude(u, ref):
    return 10 * math.log10(float(np.max(np.abs(ref))) / float(np.mean(np.abs(u - ref))))


def _psnr_sum_not_mean(u, ref):
    return 10 * math.log10(float(np.max(np.abs(ref)) ** 2) / float(np.sum(np.abs(u - ref) ** 2)))


def _psnr_real_part(u, ref):
    return 10 * math.log10(float(np.max(np.abs(ref.real)) ** 2) / float(np.mean((u.real - ref.real) ** 2)))


def _rel_by_u(u, ref):
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(u.ravel()))


def _rel_squared(u, ref):
    return float(np.sum(np.abs(u - ref) ** 2) / np.sum(np.abs(ref) ** 2))


def _rel_rowwise_max(u, ref):
    d = np.atleast_2d(u - ref)
    r = np.atleast_2d(ref)
    return float(np.max(np.linalg.norm(d, axis=-1) / np.linalg.norm(r, axis=-1)))


@pytest.mark.parametrize("mutant", [_psnr_peak_from_u, _psnr_magnitude, _psnr_sum_not_mean, _psnr_real_part])
def test_planted_psnr_mistakes_fail_the_pin(mutant):
    with pytest.raises(AssertionError):
        check_psnr(mutant)


@pytest.mark.parametrize("mutant", [_rel_by_u, _rel_squared, _rel_rowwise_max])
def test_planted_rel_l2_mistakes_fail_the_pin(mutant):
    with pytest.raises(AssertionError):
        check_rel_l2(mutant)
