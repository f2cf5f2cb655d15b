"""Pins for the oracle's Eq.(1) direct sum and its circ() window (Sec. 2, step 1)."""
import numpy as np

from conftest import read_golden

P = 1e-6


def _jacobi_r2(n):
    """Number of integer pairs (x, y) with x^2 + y^2 = n (Jacobi's two-square theorem)."""
    if n == 0:
        return 1
    s = 0
    for d in range(1, n + 1):
        if n % d == 0 and d % 2 == 1:
            s += 1 if d % 4 == 1 else -1
    return 4 * s


def test_pythagorean_pixels_full_and_circ(orc):
    (rows,) = read_golden("direct_pythagorean.txt")
    lam = 0.8e-6
    pts = np.array([[0.0, 0.0, 12e-6, 0.7]])
    for window in (orc.FULL, orc.CIRC):
        u = orc.direct(pts, nx=20, ny=20, ox=0, oy=0, pitch=P, wavelength=lam, window=window)
        for dx, dy, re, im, inside in rows:
            expect = complex(re, im) if (window == orc.FULL or inside) else 0.0
            assert abs(u[int(dy), int(dx)] - expect) < 1e-12, (dx, dy, window)


def test_circ_support_is_gauss_lattice_count(orc):
    # R^2 = (z tan theta / p)^2 chosen between 10 and 11: the disk holds sum_{n<=10} r2(n) pixels.
    lam = 633e-9
    s = lam / (2 * P)
    tan_t = s / np.sqrt(1 - s * s)
    z = 3.2 * P / tan_t                      # R = 3.2 px, R^2 = 10.24
    pts = np.array([[16 * P, 16 * P, z, 1.0]])
    u = orc.direct(pts, nx=32, ny=32, pitch=P, wavelength=lam, window=orc.CIRC)
    expect = sum(_jacobi_r2(n) for n in range(11))
    assert expect == 37
    assert int(np.count_nonzero(u)) == expect
    full = orc.direct(pts, nx=32, ny=32, pitch=P, wavelength=lam, window=orc.FULL)
    np.testing.assert_allclose(np.abs(full), 1.0, atol=1e-12)
    mask = u != 0
    np.testing.assert_array_equal(u[mask], full[mask])


def test_circ_boundary_is_strict(orc):
    """circ(c) = 1 only for c < 1 (Sec. 2, step 1): a pixel exactly on the PSF's rim is outside.
    With pitch 1 and lambda 1.2 (any unit), tan(theta) = 0.75 and z = 5 / tan(theta) make
    R^2 = 25 exactly in FP64, so the 12 pixels at squared distance 25 (offsets (+-3, +-4),
    (+-4, +-3), (+-5, 0), (0, +-5)) lie on the rim: the disk holds sum_{n<25} r2(n) = 69 pixels."""
    p, lam = 1.0, 1.2
    s = lam / (2.0 * p)
    tan_t = s / np.sqrt(1.0 - s * s)
    z = 5.0 / tan_t
    assert (z * tan_t) * (z * tan_t) == 25.0          # the rim is hit exactly in FP64
    pts = np.array([[8.0, 8.0, z, 1.0]])
    u = orc.direct(pts, nx=17, ny=17, pitch=p, wavelength=lam, window=orc.CIRC)
    inside = sum(_jacobi_r2(n) for n in range(25))
    assert inside == 69 and _jacobi_r2(25) == 12
    assert int(np.count_nonzero(u)) == inside
    for dx, dy in ((3, 4), (4, -3), (-5, 0), (0, 5)):
        assert u[8 + dy, 8 + dx] == 0
    assert abs(u[8 + 4, 8 + 2]) > 0.5                  # squared distance 20, inside
    # the pre-computed PSF table draws the same rim: R = 5 exactly, the same 69 pixels
    T = orc.psf_table(z, 5.0, 16, pitch=p, wavelength=lam)
    assert int(np.count_nonzero(T)) == inside


def test_linearity_in_amplitude(orc):
    rng = np.random.default_rng(1)
    pts = np.stack([rng.uniform(0, 24e-6, 5), rng.uniform(0, 24e-6, 5),
                    rng.uniform(20e-6, 60e-6, 5), rng.uniform(0, 1, 5)], axis=1)
    whole = orc.direct(pts, 24, 24, window=orc.CIRC)
    parts = sum(orc.direct(pts[k:k + 1], 24, 24, window=orc.CIRC) for k in range(5))
    np.testing.assert_allclose(whole, parts, atol=1e-12)
    scaled = pts.copy()
    scaled[:, 3] *= 3.0
    np.testing.assert_allclose(orc.direct(scaled, 24, 24), 3.0 * orc.direct(pts, 24, 24), atol=1e-12)


def test_translation_and_transpose(orc):
    rng = np.random.default_rng(2)
    pts = np.stack([rng.uniform(0, 30e-6, 7), rng.uniform(0, 20e-6, 7),
                    rng.uniform(30e-6, 80e-6, 7), rng.uniform(0, 1, 7)], axis=1)
    u = orc.direct(pts, nx=30, ny=20, ox=0, oy=0)
    moved = pts.copy()
    moved[:, 0] += 5 * P
    moved[:, 1] -= 9 * P
    v = orc.direct(moved, nx=30, ny=20, ox=5, oy=-9)
    np.testing.assert_allclose(v, u, atol=1e-9)
    swapped = pts[:, [1, 0, 2, 3]]
    t = orc.direct(swapped, nx=20, ny=30)
    np.testing.assert_array_equal(t, u.T)
    # a rectangular window picks the right rows and columns
    w = orc.direct(pts, nx=7, ny=5, ox=11, oy=3)
    np.testing.assert_array_equal(w, u[3:8, 11:18])
