"""Pins for the oracle's angular-spectrum propagation (numerical reconstruction, Sec. 3) and its
wavefront-recording-plane composition.

* a plane wave on the FFT grid stays a plane wave and gains exactly the phase
  2 pi d sqrt(1/lambda^2 - fx^2 - fy^2) (closed form; catches a wrong sign, scale or axis);
* components beyond 1/lambda (possible with a pitch below lambda / 2) are dropped;
* propagating by d and then by -d gives the field back; d1 then d2 equals d1 + d2;
* energy is kept (Parseval) for fields without evanescent components;
* the WRP hologram of points on the WRP's grid is WASABI's hologram on the WRP, propagated.
"""
import numpy as np
import pytest

from workloads import grid_points

LAM, P = 633e-9, 1e-6


def _plane(nx, ny, a, b, pitch=P):
    x = np.arange(nx) * pitch
    y = np.arange(ny) * pitch
    fx, fy = a / (nx * pitch), b / (ny * pitch)
    return np.exp(2j * np.pi * (fx * x[None, :] + fy * y[:, None])), fx, fy


@pytest.mark.parametrize("a,b,d", [(3, -5, 200e-6), (-31, 0, -1.5e-3), (0, 0, 7e-3), (12, 20, 25e-6)])
def test_plane_wave_gains_the_closed_form_phase(orc, a, b, d):
    u, fx, fy = _plane(64, 48, a, b)
    out = orc.propagate(u, d)
    phase = 2 * np.pi * d * np.sqrt(1 / LAM ** 2 - fx ** 2 - fy ** 2)
    np.testing.assert_allclose(out, u * np.exp(1j * phase), atol=1e-11)


def test_evanescent_components_are_dropped(orc):
    pitch = 0.25e-6                                # |f| up to 2 / um > 1 / lambda
    u, fx, fy = _plane(32, 32, 13, 0, pitch)       # fx = 1.625 / um > 1 / 0.633 um
    assert fx > 1 / LAM
    assert np.abs(orc.propagate(u, 1e-6, pitch=pitch)).max() < 1e-12
    v, _, _ = _plane(32, 32, 5, 0, pitch)          # fx = 0.625 / um propagates
    assert np.abs(orc.propagate(v, 1e-6, pitch=pitch)).min() > 1 - 1e-12


def test_round_trip_composition_and_energy(orc):
    rng = np.random.default_rng(3)
    u = rng.normal(size=(96, 128)) + 1j * rng.normal(size=(96, 128))
    f = orc.propagate(u, 0.8e-3)
    np.testing.assert_allclose(orc.propagate(f, -0.8e-3), u, atol=1e-10)
    np.testing.assert_allclose(orc.propagate(orc.propagate(u, 0.3e-3), 0.5e-3), f, atol=1e-10)
    assert abs(np.linalg.norm(f) / np.linalg.norm(u) - 1) < 1e-12


def test_wrp_is_wasabi_on_the_plane_then_propagation(orc):
    prm = orc.LutParams(z_min=20e-6, z_max=70e-6, n_depth=4, levels=3, gamma=0.3, max_window=128,
                        value_dtype=3)
    lut = orc.build_lut(prm)
    z_wrp = 1.0e-3
    pts = grid_points(5, 20, 128, 96, 8, 20e-6 + z_wrp, 70e-6 + z_wrp)
    u = orc.wrp(lut, pts, z_wrp, 128, 96)
    rel = pts.copy()
    rel[:, 2] -= z_wrp
    on_plane = orc.wasabi(lut, orc.quantize(rel, prm), 0, 0, 128, 96)
    np.testing.assert_allclose(orc.propagate(u, -z_wrp), on_plane, atol=1e-10)
    assert np.linalg.norm(on_plane) > 1.0
