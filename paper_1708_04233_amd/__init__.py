"""Python binding of libcgh.so, the MI355X (gfx950) WASABI hologram library.

Argument marshalling only: every step runs in the library's HIP kernels.  Tensors are torch
tensors on the current HIP device; calls run on ``torch.cuda.current_stream()``.  The names follow
the C ABI in ``include/cgh.h``:

  cgh_direct              Eq.(1), direct superposition (FULL or CIRC window)
  wasabi_build_lut        Sec. 2 step 1, PSF tables -> Haar -> N_r strongest coefficients
  wasabi_lut_import       the same LUT object from canonical host arrays
  wasabi_quantize         depth planes and the 2^L position grid
  wasabi_superpose        Eq.(2) on one sub-hologram, wavelet field in Mallat layout
  wasabi_idwt             inverse Haar transform (Sec. 2 step 3)
  wasabi_hologram         sub-hologram procedure (Sec. 2, large-scale steps 2-4)
  wasabi_hologram_fused   the same, tile by tile in on-chip memory
  wasabi_hologram_fused_noalloc  the same without allocating (static scratch buffer)
  cgh_propagate           angular-spectrum propagation (numerical reconstruction)
  wasabi_hologram_wrp     WASABI on a wavefront recording plane, then propagation
  Server                  cgh_server_*: hologram jobs with continuous batching under a memory budget
"""
from __future__ import annotations

import ctypes
import os
import re
from dataclasses import dataclass

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcgh.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "cgh.h")

CGH_OK, CGH_EINVAL, CGH_ENOMEM, CGH_EHIP, CGH_EAGAIN = 0, -1, -2, -3, -4
CGH_ENOTFOUND, CGH_ETIMEDOUT, CGH_ECANCELED = -5, -6, -7
C64, C128 = 0, 1
F32, F16, BF16 = 0, 1, 2
FULL, CIRC = 0, 1
HAAR, COIF1 = 0, 1


class CghError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("cgh error %d: %s" % (code, msg))
        self.code = code


class _LutParams(ctypes.Structure):
    _fields_ = [("wavelength", ctypes.c_double), ("pitch", ctypes.c_double),
                ("z_min", ctypes.c_double), ("z_max", ctypes.c_double),
                ("n_depth", ctypes.c_int32), ("levels", ctypes.c_int32),
                ("max_window", ctypes.c_int32), ("value_dtype", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("phases", ctypes.c_int32), ("wavelet", ctypes.c_int32)]


class _ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("max_slots", ctypes.c_int32),
                ("simulate", ctypes.c_int32), ("sim_ns_per_pixel", ctypes.c_double),
                ("lut", ctypes.c_void_p), ("fail_ticket", ctypes.c_uint64)]


class _Job(ctypes.Structure):
    _fields_ = [("host_pts", ctypes.c_void_p), ("n", ctypes.c_int64), ("nx", ctypes.c_int32),
                ("ny", ctypes.c_int32)]


class _Result(ctypes.Structure):
    _fields_ = [("u", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_start", ctypes.c_double), ("t_done", ctypes.c_double),
                ("gpu_ms", ctypes.c_double), ("status", ctypes.c_int32), ("slot", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("canceled", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("queued", ctypes.c_int64), ("running", ctypes.c_int64),
                ("max_running", ctypes.c_int64), ("bytes_in_use", ctypes.c_size_t),
                ("peak_bytes", ctypes.c_size_t), ("arena_bytes", ctypes.c_size_t),
                ("lut_bytes", ctypes.c_size_t)]


_lib = None


def load() -> ctypes.CDLL:
    """Load the in-tree libcgh.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcgh.so is not built (run `python paper_1708_04233_amd/build.py`)")
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, D = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "cgh_last_error": ([], ctypes.c_char_p),
        "cgh_direct": ([P, I64, I32, I32, I64, I64, D, D, I32, I32, P, I64, P], ctypes.c_int),
        "wasabi_build_lut": ([ctypes.POINTER(_LutParams), ctypes.POINTER(P), P], ctypes.c_int),
        "wasabi_lut_import": ([ctypes.POINTER(_LutParams), P, P, P, ctypes.POINTER(P)], ctypes.c_int),
        "wasabi_lut_info": ([P, P, P, P, P, P, P, P], ctypes.c_int),
        "wasabi_lut_export": ([P, P, P, P], ctypes.c_int),
        "wasabi_lut_free": ([P], None),
        "wasabi_quantize": ([P, P, I64, P, P], ctypes.c_int),
        "wasabi_superpose": ([P, P, I64, I64, I64, I32, I32, P, I32, P], ctypes.c_int),
        "wasabi_idwt": ([P, I32, I32, I32, P, I64, P], ctypes.c_int),
        "wasabi_hologram": ([P, P, I64, I64, I64, I32, I32, I32, P, I64, P], ctypes.c_int),
        "wasabi_hologram_fused": ([P, P, I64, I64, I64, I32, I32, P, I64, P], ctypes.c_int),
        "wasabi_hologram_fused_noalloc": ([P, P, I64, I64, I64, I32, I32, P, I64, P], ctypes.c_int),
        "cgh_propagate": ([P, P, I32, I32, D, D, D, P], ctypes.c_int),
        "wasabi_hologram_wrp": ([P, P, I64, D, I32, I32, P, P], ctypes.c_int),
        "cgh_server_create": ([ctypes.POINTER(_ServerConfig), ctypes.POINTER(P)], ctypes.c_int),
        "cgh_server_submit": ([P, ctypes.POINTER(_Job), ctypes.POINTER(ctypes.c_uint64)], ctypes.c_int),
        "cgh_server_wait": ([P, ctypes.c_uint64, I32, ctypes.POINTER(_Result)], ctypes.c_int),
        "cgh_server_cancel": ([P, ctypes.c_uint64], ctypes.c_int),
        "cgh_server_release": ([P, ctypes.c_uint64], ctypes.c_int),
        "cgh_server_query": ([P, ctypes.POINTER(_Stats)], ctypes.c_int),
        "cgh_server_destroy": ([P], ctypes.c_int),
        "cgh_profile_enable": ([I32], ctypes.c_int),
        "cgh_profile_reset": ([], ctypes.c_int),
        "cgh_profile_query": ([ctypes.c_char_p, ctypes.POINTER(D), ctypes.POINTER(I64)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    _lib = lib
    return lib


def header_functions() -> list:
    """Names of the functions declared in include/cgh.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", text)) -
                  {"if", "while", "for", "return", "sizeof"})


def _check(rc: int):
    if rc != CGH_OK:
        raise CghError(rc, load().cgh_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None, shape=None):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise ValueError("%s must be a tensor on the GPU" % name)
    if dtype is not None and t.dtype != dtype:
        raise ValueError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s, got %s" % (name, shape, tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


def cgh_profile_enable(on: bool = True):
    _check(load().cgh_profile_enable(1 if on else 0))


def cgh_profile_reset():
    _check(load().cgh_profile_reset())


def cgh_profile_query(name: str):
    """(total milliseconds, launches) recorded for kernel group `name` since the last reset."""
    t = ctypes.c_double()
    k = ctypes.c_int64()
    _check(load().cgh_profile_query(name.encode(), ctypes.byref(t), ctypes.byref(k)))
    return t.value, k.value


# ----------------------------------------------------------------------------------------------
def cgh_direct(pts: torch.Tensor, nx: int, ny: int, ox: int = 0, oy: int = 0,
               pitch: float = 1e-6, wavelength: float = 633e-9, window: int = FULL,
               out: torch.Tensor | None = None, out_dtype=torch.complex64) -> torch.Tensor:
    """Eq.(1) on the ny x nx window at global pixel (ox, oy); pts (n, 4) float64 {x, y, z, a}."""
    n = pts.shape[0]
    if out is None:
        out = torch.empty((ny, nx), dtype=out_dtype, device=pts.device)
    if out.dim() != 2 or out.shape[1] < nx or out.shape[0] != ny or out.stride(1) != 1:
        raise ValueError("out must be (ny, >=nx) with unit column stride")
    code = {torch.complex64: C64, torch.complex128: C128}[out.dtype]
    pp = _dev(pts, "pts", torch.float64, (n, 4))
    _check(load().cgh_direct(pp, n, nx, ny, ox, oy, pitch, wavelength, window, code,
                             ctypes.c_void_p(out.data_ptr()), out.stride(0), _stream()))
    return out


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
    phases: int = 0   # 1: 4^L phase tables per plane, points on any pixel
    wavelet: int = HAAR  # COIF1: the coiflet of order 1 (holograms through wasabi_hologram)

    def c(self) -> _LutParams:
        return _LutParams(self.wavelength, self.pitch, self.z_min, self.z_max, self.n_depth,
                          self.levels, self.max_window, self.value_dtype, self.gamma,
                          int(self.phases), int(self.wavelet))


class Lut:
    """Device-resident coefficient LUT (owns the library handle)."""

    def __init__(self, handle: ctypes.c_void_p, params: LutParams):
        self.handle = handle
        self.params = params

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.wasabi_lut_free(self.handle)
            self.handle = None

    def info(self) -> dict:
        lib = load()
        nd = ctypes.c_int32()
        tot = ctypes.c_int64()
        dev_bytes = ctypes.c_int64()
        _check(lib.wasabi_lut_info(self.handle, ctypes.byref(nd), ctypes.byref(tot),
                                   ctypes.byref(dev_bytes), None, None, None, None))
        n = nd.value
        z = np.zeros(n); R = np.zeros(n)
        W = np.zeros(n, np.int32); Nr = np.zeros(n, np.int64)
        _check(lib.wasabi_lut_info(self.handle, None, None, None, z.ctypes.data, R.ctypes.data,
                                   W.ctypes.data, Nr.ctypes.data))
        return dict(n_tables=n, total_entries=tot.value, device_bytes=dev_bytes.value, z=z, R=R,
                    W=W, Nr=Nr)

    def export(self):
        """(off, idx, val): canonical layout, val complex128 holding the stored values."""
        inf = self.info()
        tot = inf["total_entries"]
        off = np.zeros(inf["n_tables"] + 1, np.int64)
        idx = np.zeros(max(tot, 1), np.int32)
        val = np.zeros(2 * max(tot, 1))
        _check(load().wasabi_lut_export(self.handle, off.ctypes.data, idx.ctypes.data, val.ctypes.data))
        return off, idx[:tot], val.view(np.complex128)[:tot]


def wasabi_build_lut(params: LutParams) -> Lut:
    h = ctypes.c_void_p()
    prm = params.c()
    _check(load().wasabi_build_lut(ctypes.byref(prm), ctypes.byref(h), _stream()))
    return Lut(h, params)


def wasabi_lut_import(params: LutParams, off: np.ndarray, idx: np.ndarray, val: np.ndarray) -> Lut:
    off = np.ascontiguousarray(off, np.int64)
    idx = np.ascontiguousarray(idx, np.int32)
    v = np.ascontiguousarray(np.asarray(val, np.complex128)).view(np.float64)
    if idx.size == 0:
        idx = np.zeros(1, np.int32)
        v = np.zeros(2)
    h = ctypes.c_void_p()
    prm = params.c()
    torch.cuda.current_stream().synchronize()
    _check(load().wasabi_lut_import(ctypes.byref(prm), off.ctypes.data, idx.ctypes.data,
                                    v.ctypes.data, ctypes.byref(h)))
    return Lut(h, params)


def points_tensor(n: int, device="cuda") -> torch.Tensor:
    """Storage for n wasabi_point records {int32 x, y, depth; float32 a} as an (n, 4) int32 tensor."""
    return torch.empty((n, 4), dtype=torch.int32, device=device)


def point_amplitudes(q: torch.Tensor) -> torch.Tensor:
    return q[:, 3].contiguous().view(torch.float32)


def wasabi_quantize(lut: Lut, pts: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    n = pts.shape[0]
    if out is None:
        out = points_tensor(n, pts.device)
    pp = _dev(pts, "pts", torch.float64, (n, 4))
    _check(load().wasabi_quantize(lut.handle, pp, n, _dev(out, "out", torch.int32, (n, 4)), _stream()))
    return out


def wasabi_superpose(lut: Lut, q: torch.Tensor, ox: int, oy: int, nx: int, ny: int,
                     psi: torch.Tensor | None = None, accumulate: bool = False) -> torch.Tensor:
    """Eq.(2) into psi (Mallat layout); accumulate=True adds to the values psi already holds."""
    n = q.shape[0]
    if psi is None:
        if accumulate:
            raise ValueError("accumulate needs psi")
        psi = torch.empty((ny, nx), dtype=torch.complex64, device=q.device)
    _check(load().wasabi_superpose(lut.handle, _dev(q, "points", torch.int32, (n, 4)), n, ox, oy,
                                   nx, ny, _dev(psi, "psi", torch.complex64, (ny, nx)),
                                   1 if accumulate else 0, _stream()))
    return psi


def wasabi_idwt(psi: torch.Tensor, levels: int, u: torch.Tensor | None = None) -> torch.Tensor:
    """Inverse Haar of the Mallat field psi into u; u may be psi itself (in place)."""
    ny, nx = psi.shape
    if u is None:
        u = torch.empty((ny, nx), dtype=torch.complex64, device=psi.device)
    if u.dtype != torch.complex64 or u.dim() != 2 or u.shape[0] != ny or u.shape[1] < nx or u.stride(1) != 1:
        raise ValueError("u must be complex64 (ny, >=nx) with unit column stride")
    _check(load().wasabi_idwt(_dev(psi, "psi", torch.complex64), nx, ny, levels,
                              ctypes.c_void_p(u.data_ptr()), u.stride(0), _stream()))
    return u


def _out_window(u, nx, ny, device):
    if u is None:
        u = torch.empty((ny, nx), dtype=torch.complex64, device=device)
    if u.dtype != torch.complex64 or u.dim() != 2 or u.shape[0] != ny or u.shape[1] < nx or u.stride(1) != 1:
        raise ValueError("u must be complex64 (ny, >=nx) with unit column stride")
    return u


def wasabi_hologram(lut: Lut, q: torch.Tensor, ox: int, oy: int, nx: int, ny: int, sub: int = 0,
                    u: torch.Tensor | None = None) -> torch.Tensor:
    n = q.shape[0]
    u = _out_window(u, nx, ny, q.device)
    _check(load().wasabi_hologram(lut.handle, _dev(q, "points", torch.int32, (n, 4)), n, ox, oy,
                                  nx, ny, sub, ctypes.c_void_p(u.data_ptr()), u.stride(0), _stream()))
    return u


def wasabi_hologram_fused(lut: Lut, q: torch.Tensor, ox: int, oy: int, nx: int, ny: int,
                          u: torch.Tensor | None = None) -> torch.Tensor:
    n = q.shape[0]
    u = _out_window(u, nx, ny, q.device)
    _check(load().wasabi_hologram_fused(lut.handle, _dev(q, "points", torch.int32, (n, 4)), n, ox,
                                        oy, nx, ny, ctypes.c_void_p(u.data_ptr()), u.stride(0),
                                        _stream()))
    return u


def wasabi_hologram_fused_noalloc(lut: Lut, q: torch.Tensor, ox: int, oy: int, nx: int, ny: int,
                                  u: torch.Tensor) -> torch.Tensor:
    """wasabi_hologram_fused with the library's static scratch buffer: allocates nothing."""
    n = q.shape[0]
    u = _out_window(u, nx, ny, q.device)
    _check(load().wasabi_hologram_fused_noalloc(lut.handle, _dev(q, "points", torch.int32, (n, 4)), n, ox,
                                                oy, nx, ny, ctypes.c_void_p(u.data_ptr()), u.stride(0),
                                                _stream()))
    return u


def cgh_propagate(u: torch.Tensor, distance: float, pitch: float = 1e-6, wavelength: float = 633e-9,
                  out: torch.Tensor | None = None) -> torch.Tensor:
    """Angular-spectrum propagation of the complex64 field u (ny, nx) by `distance` metres."""
    ny, nx = u.shape
    _dev(u, "u", torch.complex64)
    out = torch.empty_like(u) if out is None else out
    _dev(out, "out", torch.complex64, (ny, nx))
    _check(load().cgh_propagate(ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(out.data_ptr()), nx, ny,
                                distance, pitch, wavelength, _stream()))
    return out


def wasabi_hologram_wrp(lut: Lut, pts: torch.Tensor, z_wrp: float, nx: int, ny: int,
                        u: torch.Tensor | None = None) -> torch.Tensor:
    """Hologram through a wavefront recording plane z_wrp metres away; pts (n, 4) float64 on the GPU."""
    n = pts.shape[0]
    u = torch.empty((ny, nx), dtype=torch.complex64, device=pts.device) if u is None else u
    _dev(u, "u", torch.complex64, (ny, nx))
    _check(load().wasabi_hologram_wrp(lut.handle, _dev(pts, "pts", torch.float64, (n, 4)), n, z_wrp, nx, ny,
                                      ctypes.c_void_p(u.data_ptr()), _stream()))
    return u


class _DeviceArray:
    """A device buffer owned by the library, seen by torch through __cuda_array_interface__."""

    def __init__(self, ptr: int, shape):
        self.__cuda_array_interface__ = {"shape": tuple(shape), "typestr": "<f4", "data": (ptr, False),
                                         "version": 2, "strides": None}


class Server:
    """cgh_server_*: a queue of hologram jobs (host points -> ny x nx complex64 hologram) served with
    continuous batching on `max_slots` streams under a device-memory budget.  simulate=True models
    the schedule on the host only (no device work; results carry no hologram)."""

    def __init__(self, lut: Lut | None, hbm_budget_bytes: int, max_slots: int = 2,
                 simulate: bool = False, sim_ns_per_pixel: float = 0.0, fail_ticket: int = 0):
        self._lut = lut  # keeps the LUT alive while the server exists
        cfg = _ServerConfig(hbm_budget_bytes, max_slots, 1 if simulate else 0, sim_ns_per_pixel,
                            lut.handle if lut is not None else None, fail_ticket)
        h = ctypes.c_void_p()
        _check(load().cgh_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def submit(self, pts: np.ndarray | None, nx: int, ny: int) -> int:
        """Queue one hologram of the (n, 4) float64 host points {x, y, z, a} (metres); returns the ticket."""
        if pts is None:
            pts = np.zeros((0, 4))
        pts = np.ascontiguousarray(pts, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 4:
            raise ValueError("pts must be (n, 4)")
        job = _Job(pts.ctypes.data if len(pts) else None, len(pts), nx, ny)
        t = ctypes.c_uint64()
        _check(load().cgh_server_submit(self.handle, ctypes.byref(job), ctypes.byref(t)))
        return t.value

    def wait(self, ticket: int, timeout_ms: int = -1) -> dict:
        """Wait for a job; returns its times, status and (if done) the hologram as a torch view of the
        server's buffer, valid until release()."""
        r = _Result()
        _check(load().cgh_server_wait(self.handle, ticket, timeout_ms, ctypes.byref(r)))
        u = None
        if r.u:
            u = torch.view_as_complex(torch.as_tensor(_DeviceArray(r.u, (r.ny, r.nx, 2)), device="cuda"))
        return {"u": u, "nx": r.nx, "ny": r.ny, "t_submit": r.t_submit, "t_admit": r.t_admit,
                "t_start": r.t_start, "t_done": r.t_done, "gpu_ms": r.gpu_ms, "status": r.status,
                "slot": r.slot}

    def cancel(self, ticket: int):
        _check(load().cgh_server_cancel(self.handle, ticket))

    def release(self, ticket: int):
        """Give the job's result back.  Work that torch queued on the current stream (a clone of the
        result, say) may still read it, and the server may hand the memory to its next job at once,
        so that stream is synchronised first (when torch has touched the GPU at all)."""
        if torch.cuda.is_initialized():
            torch.cuda.current_stream().synchronize()
        _check(load().cgh_server_release(self.handle, ticket))

    def stats(self) -> dict:
        st = _Stats()
        _check(load().cgh_server_query(self.handle, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in _Stats._fields_}

    def close(self):
        if self.handle:
            _check(load().cgh_server_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
