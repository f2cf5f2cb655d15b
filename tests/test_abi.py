"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function that
include/cgh.h declares, and rejects bad arguments before touching the device."""
import ctypes

import pytest

import paper_1708_04233_amd as cgh


def test_exports_every_declared_function():
    lib = cgh.load()
    names = cgh.header_functions()
    assert "cgh_direct" in names and "wasabi_superpose" in names and len(names) >= 12
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []


def test_argument_validation_without_device():
    lib = cgh.load()
    out = ctypes.c_void_p(16)
    # bad sizes, wavelength >= 2 pitch, unknown window / dtype
    assert lib.cgh_direct(None, 0, 0, 4, 0, 0, 1e-6, 633e-9, 0, 0, out, 4, None) == cgh.CGH_EINVAL
    assert lib.cgh_direct(None, 0, 4, 4, 0, 0, 1e-6, 2.5e-6, 0, 0, out, 4, None) == cgh.CGH_EINVAL
    assert lib.cgh_direct(None, 0, 4, 4, 0, 0, 1e-6, 633e-9, 7, 0, out, 4, None) == cgh.CGH_EINVAL
    assert lib.cgh_direct(None, 0, 4, 4, 0, 0, 1e-6, 633e-9, 0, 9, out, 4, None) == cgh.CGH_EINVAL
    assert lib.cgh_direct(None, 3, 4, 4, 0, 0, 1e-6, 633e-9, 0, 0, out, 4, None) == cgh.CGH_EINVAL
    assert b"NULL" in lib.cgh_last_error()
    h = ctypes.c_void_p()
    for bad in [dict(levels=0), dict(levels=7), dict(n_depth=0), dict(gamma=0.0),
                dict(z_min=2e-3), dict(wavelength=3e-6), dict(value_dtype=5),
                dict(max_window=512), dict(phases=2), dict(phases=1, n_depth=65536),
                dict(phases=1, levels=5),    # phase tables: 2 * 496 + 64 > 1024
                dict(wavelet=2), dict(wavelet=1, levels=5)]:   # coiflet: 2 * 496 + 2 + 320 > 1024
        prm = cgh.LutParams(**bad).c()
        assert lib.wasabi_build_lut(ctypes.byref(prm), ctypes.byref(h), None) == cgh.CGH_EINVAL, bad
        assert not h.value
    assert lib.wasabi_idwt(out, 12, 16, 3, out, 16, None) == cgh.CGH_EINVAL   # 12 % 8 != 0
    # u overlapping psi other than as the same contiguous array (in place needs u == psi, ld == nx)
    shifted = ctypes.c_void_p(16 + 8 * 3)
    assert lib.wasabi_idwt(out, 16, 16, 3, shifted, 16, None) == cgh.CGH_EINVAL
    assert lib.wasabi_idwt(out, 16, 16, 3, out, 24, None) == cgh.CGH_EINVAL
    assert b"overlap" in lib.cgh_last_error()
    assert lib.wasabi_superpose(None, None, 0, 0, 0, 16, 16, out, 0, None) == cgh.CGH_EINVAL
    assert lib.wasabi_superpose(None, None, 0, 0, 0, 16, 16, out, 2, None) == cgh.CGH_EINVAL
    # propagation: NULL field, sides not powers of two or beyond 8192, bad pitch / distance
    assert lib.cgh_propagate(None, out, 64, 64, 1e-3, 1e-6, 633e-9, None) == cgh.CGH_EINVAL
    assert lib.cgh_propagate(out, out, 96, 64, 1e-3, 1e-6, 633e-9, None) == cgh.CGH_EINVAL
    assert lib.cgh_propagate(out, out, 64, 16384, 1e-3, 1e-6, 633e-9, None) == cgh.CGH_EINVAL
    assert lib.cgh_propagate(out, out, 64, 64, 1e-3, 0.0, 633e-9, None) == cgh.CGH_EINVAL
    assert lib.cgh_propagate(out, out, 64, 64, float("inf"), 1e-6, 633e-9, None) == cgh.CGH_EINVAL
    assert lib.wasabi_hologram_wrp(None, None, 0, 1e-3, 64, 64, out, None) == cgh.CGH_EINVAL


def test_lut_offsets_beyond_int32_rejected_before_allocation():
    """The superposition addresses kept entries and per-block offsets with 32-bit integers, so a
    LUT whose tables hold 2^30 or more Haar blocks is refused while the geometry is computed, before
    any device memory is requested (no GPU here: an allocation attempt would fail differently).
    Here 16384 planes x 64 phase tables of up to 1008^2 pixels make ~1.7e10 blocks of 8 x 8, while
    gamma = 0.001 keeps only ~8e8 entries."""
    lib = cgh.load()
    h = ctypes.c_void_p()
    prm = cgh.LutParams(n_depth=16384, levels=3, phases=1, gamma=0.001, max_window=1024).c()
    assert lib.wasabi_build_lut(ctypes.byref(prm), ctypes.byref(h), None) == cgh.CGH_EINVAL
    assert b"2^30" in lib.cgh_last_error() and b"blocks" in lib.cgh_last_error()
    assert not h.value
    # too many kept coefficients: 8192 planes of 80^2 .. 1008^2 pixels (~3e9 in all), all kept
    prm = cgh.LutParams(n_depth=8192, levels=3, gamma=1.0, max_window=1024).c()
    assert lib.wasabi_build_lut(ctypes.byref(prm), ctypes.byref(h), None) == cgh.CGH_EINVAL
    assert b"2^31" in lib.cgh_last_error() and b"coefficients" in lib.cgh_last_error()
    assert not h.value
