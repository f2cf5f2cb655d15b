"""FP64 CPU oracle for the WASABI hologram path (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may import
this package.  It shares no code with the HIP library: the arithmetic lives in ``oracle.c``
(plain loops, FP64), and this module only marshals numpy arrays into it.

Paper: Shimobaba et al., "Fast, large-scale hologram calculation in wavelet domain".
  * ``direct``          -- Eq.(1), optionally restricted to the PSF's circ() support.
  * ``lut_geometry``    -- Sec. 2 step 1 (planes, PSF radius, N_r = gamma*pi*R^2).
  * ``psf_table``       -- Sec. 2 step 1 (u_z = exp(ikr) circ(.)).
  * ``haar_forward`` / ``haar_inverse`` -- Sec. 2 steps 1 and 3, Fig. 2(a) layout (Haar wavelet).
  * ``dwt_forward`` / ``dwt_inverse``   -- the same for the coiflet the paper names (periodised).
  * ``build_lut``       -- Sec. 2 step 1 (transform + keep the N_r strongest coefficients).
  * ``quantize``        -- depth discretisation and the 2^L grid that Eq.(2) needs (or, with
                           phase tables, the pixel grid and the table of the point's phase).
  * ``superpose``       -- Eq.(2) with the sub-hologram shift of the large-scale procedure.
  * ``wasabi``          -- superpose followed by the inverse transform (Sec. 2 steps 2-4).
  * ``propagate``       -- angular-spectrum propagation of a sampled field (numerical
                           reconstruction, Sec. 3, and the wavefront-recording-plane method the
                           conclusion names as the next step); numpy's FFT is the library step.
  * ``wrp``             -- WASABI on a wavefront recording plane, then propagation to the hologram.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# The test of the pins themselves (tests/test_oracle_mutations.py) runs the pin suite against
# copies of oracle.c compiled with one planted mistake each, named by this variable.
_LIB_OVERRIDE = os.environ.get("ORACLE_LIB_OVERRIDE")
_lib = None

F32, F16, BF16, F64 = 0, 1, 2, 3
FULL, CIRC = 0, 1
HAAR, COIF1 = 0, 1


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain C, FP64, OpenMP over output rows)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if _LIB_OVERRIDE:
        lib = ctypes.CDLL(_LIB_OVERRIDE)
    else:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oracle_direct.argtypes = [P, I64, I32, I32, I64, I64, D, D, I32, P]
    lib.oracle_direct.restype = None
    lib.oracle_lut_geometry.argtypes = [D, D, D, D, I32, I32, I32, D, I32, I32, P, P, P, P]
    lib.oracle_lut_geometry.restype = ctypes.c_int
    lib.oracle_psf_table.argtypes = [D, D, I32, I32, I32, D, D, P]
    lib.oracle_psf_table.restype = None
    lib.oracle_haar_forward.argtypes = [P, I32, I32, I32]
    lib.oracle_haar_forward.restype = None
    lib.oracle_haar_inverse.argtypes = [P, I32, I32, I32]
    lib.oracle_haar_inverse.restype = None
    lib.oracle_select.argtypes = [P, I32, I64, P, P]
    lib.oracle_select.restype = None
    lib.oracle_round_value.argtypes = [D, I32]
    lib.oracle_round_value.restype = D
    lib.oracle_build_lut.argtypes = [D, D, I32, I32, P, P, P, P, P, P, P, I32, I32, P, P]
    lib.oracle_filters.argtypes = [I32, P, P]
    lib.oracle_filters.restype = I32
    lib.oracle_dwt_forward.argtypes = [P, I32, I32, I32, I32]
    lib.oracle_dwt_forward.restype = None
    lib.oracle_dwt_inverse.argtypes = [P, I32, I32, I32, I32]
    lib.oracle_dwt_inverse.restype = None
    lib.oracle_build_lut.restype = None
    lib.oracle_quantize.argtypes = [P, I64, D, D, D, I32, I32, I32, P, P, P, P]
    lib.oracle_quantize.restype = None
    lib.oracle_superpose.argtypes = [I32, P, P, P, P, P, P, P, P, I64, I64, I64, I32, I32, P]
    lib.oracle_superpose.restype = None
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _complex_from(buf: np.ndarray, shape) -> np.ndarray:
    return buf.view(np.complex128).reshape(shape)


# ----------------------------------------------------------------------------------------------
# Eq.(1)
# ----------------------------------------------------------------------------------------------
def direct(pts: np.ndarray, nx: int, ny: int, ox: int = 0, oy: int = 0, pitch: float = 1e-6,
           wavelength: float = 633e-9, window: int = FULL) -> np.ndarray:
    """u(x_h, y_h) = sum_j a_j exp(i 2 pi r_hj / lambda) on an ny x nx window (Eq.(1)).

    pts: (n, 4) float64 {x, y, z, a}, metres.  window=CIRC restricts each point to its PSF disk.
    """
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 4)
    out = np.zeros(2 * nx * ny, dtype=np.float64)
    lib.oracle_direct(_p(pts), pts.shape[0], nx, ny, ox, oy, pitch, wavelength, window, _p(out))
    return _complex_from(out, (ny, nx))


# ----------------------------------------------------------------------------------------------
# LUT (Sec. 2, step 1)
# ----------------------------------------------------------------------------------------------
@dataclass
class LutParams:
    wavelength: float = 633e-9
    pitch: float = 1e-6
    z_min: float = 0.1e-3
    z_max: float = 1.5e-3
    n_depth: int = 64
    levels: int = 3
    max_window: int = 1024
    gamma: float = 0.05
    value_dtype: int = F32
    phases: int = 0        # 1: one table per depth and position inside the 2^L block (4^L per depth)
    wavelet: int = 0       # 0: Haar; 1: the coiflet of order 1 (HAAR, COIF1)


@dataclass
class Lut:
    """Canonical LUT: table t owns entries [off[t], off[t+1]) sorted by flat table index.

    Without phase tables table t is plane t.  With them table t = d 4^L + sy 2^L + sx holds plane
    d's PSF for a point sx columns right of and sy rows below its 2^L block's corner."""
    params: LutParams
    z: np.ndarray      # (n_tables,) plane depth z_d, metres
    R: np.ndarray      # (n_tables,) PSF radius, pixels
    W: np.ndarray      # (n_tables,) table side, int32
    Nr: np.ndarray     # (n_tables,) kept coefficients, int64
    off: np.ndarray    # (n_tables + 1,) int64
    idx: np.ndarray    # (sum Nr,) int32 flat index row * W + col
    val: np.ndarray    # (sum Nr,) complex128, already rounded to the storage dtype
    sx: np.ndarray = None  # (n_tables,) disk centre shift from the table centre, columns
    sy: np.ndarray = None  # (n_tables,) rows


def n_phases(prm: LutParams) -> int:
    return 1 << (2 * prm.levels) if prm.phases else 1


def lut_geometry(prm: LutParams):
    """Per table: z, R, W, N_r (planes repeated once per phase with phase tables), and the disk
    centre shifts sx, sy."""
    lib = _load()
    n = prm.n_depth
    z = np.zeros(n); R = np.zeros(n)
    W = np.zeros(n, dtype=np.int32); Nr = np.zeros(n, dtype=np.int64)
    rc = lib.oracle_lut_geometry(prm.wavelength, prm.pitch, prm.z_min, prm.z_max, n, prm.levels,
                                 prm.max_window, prm.gamma, int(prm.phases), int(prm.wavelet), _p(z), _p(R),
                                 _p(W), _p(Nr))
    if rc != 0:
        raise ValueError("a PSF table exceeds max_window")
    P, B = n_phases(prm), 1 << prm.levels
    ph = np.tile(np.arange(P, dtype=np.int32), n)
    sx = (ph % B if prm.phases else np.zeros_like(ph)).astype(np.int32)
    sy = (ph // B if prm.phases else np.zeros_like(ph)).astype(np.int32)
    return np.repeat(z, P), np.repeat(R, P), np.repeat(W, P), np.repeat(Nr, P), sx, sy


def psf_table(z: float, R: float, W: int, pitch: float = 1e-6, wavelength: float = 633e-9,
              sx: int = 0, sy: int = 0):
    lib = _load()
    out = np.zeros(2 * W * W)
    lib.oracle_psf_table(z, R, W, sx, sy, pitch, wavelength, _p(out))
    return _complex_from(out, (W, W))


def haar_forward(a: np.ndarray, levels: int) -> np.ndarray:
    lib = _load()
    b = np.ascontiguousarray(a, dtype=np.complex128).copy()
    h, w = b.shape
    lib.oracle_haar_forward(_p(b), h, w, levels)
    return b


def haar_inverse(a: np.ndarray, levels: int) -> np.ndarray:
    lib = _load()
    b = np.ascontiguousarray(a, dtype=np.complex128).copy()
    h, w = b.shape
    lib.oracle_haar_inverse(_p(b), h, w, levels)
    return b


def filters(wavelet: int):
    """(lo, hi) analysis filters: Haar, or the six-tap coiflet from its closed form."""
    lo = np.zeros(8); hi = np.zeros(8)
    taps = _load().oracle_filters(wavelet, _p(lo), _p(hi))
    return lo[:taps].copy(), hi[:taps].copy()


def dwt_forward(a: np.ndarray, levels: int, wavelet: int) -> np.ndarray:
    """Periodised orthonormal L-level 2-D transform in the Mallat layout (Haar for wavelet 0)."""
    b = np.ascontiguousarray(a, dtype=np.complex128).copy()
    h, w = b.shape
    _load().oracle_dwt_forward(_p(b), h, w, levels, wavelet)
    return b


def dwt_inverse(a: np.ndarray, levels: int, wavelet: int) -> np.ndarray:
    b = np.ascontiguousarray(a, dtype=np.complex128).copy()
    h, w = b.shape
    _load().oracle_dwt_inverse(_p(b), h, w, levels, wavelet)
    return b


def halo(prm: LutParams) -> int:
    """Extra pixels around a window whose coiflet-domain field is inverted (5 2^L: the reach of
    the periodised six-tap filters over L levels); 0 for Haar, whose blocks are independent."""
    return 5 * (1 << prm.levels) if prm.wavelet == COIF1 else 0


def select(C: np.ndarray, Nr: int):
    lib = _load()
    C = np.ascontiguousarray(C, dtype=np.complex128)
    W = C.shape[0]
    idx = np.zeros(Nr, dtype=np.int32)
    val = np.zeros(2 * Nr)
    lib.oracle_select(_p(C), W, Nr, _p(idx), _p(val))
    return idx, val.view(np.complex128)


def round_value(v: float, dtype: int) -> float:
    return _load().oracle_round_value(float(v), dtype)


def build_lut(prm: LutParams) -> Lut:
    lib = _load()
    z, R, W, Nr, sx, sy = lut_geometry(prm)
    nt = len(z)
    off = np.zeros(nt + 1, dtype=np.int64)
    off[1:] = np.cumsum(Nr)
    total = int(off[-1])
    idx = np.zeros(total, dtype=np.int32)
    val = np.zeros(2 * total)
    lib.oracle_build_lut(prm.wavelength, prm.pitch, nt, prm.levels, _p(z), _p(R), _p(W),
                         _p(Nr), _p(sx), _p(sy), _p(off), prm.value_dtype, int(prm.wavelet), _p(idx), _p(val))
    return Lut(prm, z, R, W, Nr, off, idx, val.view(np.complex128), sx, sy)


# ----------------------------------------------------------------------------------------------
# Points, Eq.(2), inverse transform
# ----------------------------------------------------------------------------------------------
@dataclass
class Quantized:
    x: np.ndarray  # int32 global pixel column, multiple of 2^L (any pixel with phase tables)
    y: np.ndarray  # int32 global pixel row
    d: np.ndarray  # int32 table (plane, or plane and phase), -1 = invalid
    a: np.ndarray  # float64 amplitude


def quantize(pts: np.ndarray, prm: LutParams) -> Quantized:
    lib = _load()
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 4)
    n = pts.shape[0]
    qx = np.zeros(n, np.int32); qy = np.zeros(n, np.int32); qd = np.zeros(n, np.int32)
    qa = np.zeros(n)
    lib.oracle_quantize(_p(pts), n, prm.pitch, prm.z_min, prm.z_max, prm.n_depth, prm.levels,
                        int(prm.phases), _p(qx), _p(qy), _p(qd), _p(qa))
    return Quantized(qx, qy, qd, qa)


def snapped_points(q: Quantized, lut: Lut) -> np.ndarray:
    """Quantised points back in metres {x, y, z_d, a} for the direct sum (invalid ones dropped)."""
    ok = q.d >= 0
    p = lut.params.pitch
    return np.stack([q.x[ok] * p, q.y[ok] * p, lut.z[q.d[ok]], q.a[ok]], axis=1)


def superpose(lut: Lut, q: Quantized, X0: int, Y0: int, nx: int, ny: int) -> np.ndarray:
    lib = _load()
    psi = np.zeros(2 * nx * ny)
    vals = np.ascontiguousarray(lut.val).view(np.float64)
    x = np.ascontiguousarray(q.x, np.int32); y = np.ascontiguousarray(q.y, np.int32)
    d = np.ascontiguousarray(q.d, np.int32); a = np.ascontiguousarray(q.a, np.float64)
    lib.oracle_superpose(lut.params.levels, _p(lut.W), _p(lut.off), _p(lut.idx), _p(vals),
                         _p(x), _p(y), _p(d), _p(a), x.shape[0], X0, Y0, nx, ny, _p(psi))
    return _complex_from(psi, (ny, nx))


def wasabi(lut: Lut, q: Quantized, X0: int, Y0: int, nx: int, ny: int) -> np.ndarray:
    """Hologram window (Sec. 2 large-scale steps 2-4): Eq.(2) then the inverse transform.  With
    coiflets the coefficients reach beyond their 2^L block, so the window is grown by a halo on
    every side, superposed and inverted (periodised) as a whole, and its centre kept."""
    L = lut.params.levels
    if lut.params.wavelet == HAAR:
        return haar_inverse(superpose(lut, q, X0, Y0, nx, ny), L)
    H = halo(lut.params)
    big = dwt_inverse(superpose(lut, q, X0 - H, Y0 - H, nx + 2 * H, ny + 2 * H), L, lut.params.wavelet)
    return big[H:H + ny, H:H + nx].copy()


# ----------------------------------------------------------------------------------------------
# Quality measures (definitions of the design notes; the paper prints none)
# ----------------------------------------------------------------------------------------------
def rel_l2(u: np.ndarray, ref: np.ndarray) -> float:
    """||u - ref||_2 / ||ref||_2 over all elements (the reference in the denominator)."""
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel()))


def psnr(u: np.ndarray, ref: np.ndarray) -> float:
    """10 log10(max|ref|^2 / mean|u - ref|^2) on the complex field: the peak power of the
    reference over the mean power of the error (the paper prints no quality figure; this is the
    reading the tests and the selectivity sweep use)."""
    mse = float(np.mean(np.abs(u - ref) ** 2))
    peak = float(np.max(np.abs(ref)) ** 2)
    return float("inf") if mse == 0 else 10.0 * np.log10(peak / mse)


# ----------------------------------------------------------------------------------------------
# Numerical propagation (reconstruction, Sec. 3) and the wavefront recording plane
# ----------------------------------------------------------------------------------------------
def propagate(u: np.ndarray, distance: float, pitch: float = 1e-6, wavelength: float = 633e-9) -> np.ndarray:
    """Angular-spectrum propagation by `distance` metres (either sign) of a field sampled on a
    pitch grid, taken as periodic: u' = IFFT2(FFT2(u) H) with
    H(fx, fy) = exp(i 2 pi d sqrt(1/lambda^2 - fx^2 - fy^2)) where fx^2 + fy^2 < 1/lambda^2 and 0
    elsewhere (evanescent waves dropped); fx = k / (nx pitch) with k in FFT order.  FP64."""
    u = np.asarray(u, dtype=np.complex128)
    ny, nx = u.shape
    fx = np.fft.fftfreq(nx, d=pitch)
    fy = np.fft.fftfreq(ny, d=pitch)
    arg = 1.0 / wavelength ** 2 - (fx[None, :] ** 2 + fy[:, None] ** 2)
    prop = arg > 0
    rev = distance * np.sqrt(np.where(prop, arg, 0.0))   # phase in revolutions
    H = np.where(prop, np.exp(2j * np.pi * (rev - np.floor(rev))), 0.0)
    return np.fft.ifft2(np.fft.fft2(u) * H)


def wrp(lut: Lut, pts: np.ndarray, z_wrp: float, nx: int, ny: int) -> np.ndarray:
    """Hologram through a wavefront recording plane (WRP) z_wrp metres from the hologram: the
    points' depths are taken from the WRP (z - z_wrp, which the LUT's planes cover), WASABI
    computes the field on the WRP, and one angular-spectrum propagation over z_wrp carries it to
    the hologram plane."""
    rel = np.array(pts, dtype=np.float64, copy=True).reshape(-1, 4)
    rel[:, 2] -= z_wrp
    u_wrp = wasabi(lut, quantize(rel, lut.params), 0, 0, nx, ny)
    return propagate(u_wrp, z_wrp, lut.params.pitch, lut.params.wavelength)
