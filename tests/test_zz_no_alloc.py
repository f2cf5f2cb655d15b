"""wasabi_hologram_fused_noalloc, called through the C ABI, against wasabi_hologram_fused: the same
hologram on two calls in a row (the second on a smaller window with fewer points, so the static
scratch buffer holds the first call's lists when it starts), for the sparse kernel (fixed-point
sums: bitwise equal) and the dense kernel with plane pacing (FP32 sums in list order: within the
FP32 tolerance).  A problem whose scratch exceeds the static buffer is refused before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1708_04233_amd as cgh
from parity import assert_field
from workloads import WASABI_2048, grid_points

pytestmark = pytest.mark.gpu


def _noalloc(lut, q, ox, oy, nx, ny, u):
    """The new entry point through ctypes on torch's current stream."""
    lib = cgh.load()
    rc = lib.wasabi_hologram_fused_noalloc(lut.handle, ctypes.c_void_p(q.data_ptr()), q.shape[0], ox, oy, nx, ny,
                                           ctypes.c_void_p(u.data_ptr()), u.stride(0),
                                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc


@pytest.mark.parametrize("gamma", [0.05, 0.84])
def test_noalloc_equals_fused_two_calls(gamma):
    w = WASABI_2048
    lut = cgh.wasabi_build_lut(cgh.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=gamma,
                                             max_window=w["max_window"]))
    calls = [(w["nx"], w["ny"], 0, 0, grid_points(w["seed"], w["n"], w["nx"], w["ny"], 8, w["z_lo"], w["z_hi"])),
             (640, 384, -256, 128, grid_points(5, 1500, 1024, 768, 8, w["z_lo"], w["z_hi"], x0=-448, y0=-64))]
    for k, (nx, ny, ox, oy, pts) in enumerate(calls):
        q = cgh.wasabi_quantize(lut, torch.from_numpy(pts).cuda())
        want = cgh.wasabi_hologram_fused(lut, q, ox, oy, nx, ny)
        got = torch.full((ny, nx + 3), complex(4.0, 4.0), dtype=torch.complex64, device="cuda")
        assert _noalloc(lut, q, ox, oy, nx, ny, got[:, :nx]) == cgh.CGH_OK, cgh.load().cgh_last_error()
        torch.cuda.synchronize()
        g = got.cpu().numpy()
        assert np.all(g[:, nx:] == complex(4.0, 4.0)), k     # nothing beyond the window's columns
        if gamma < 0.35:
            assert np.array_equal(g[:, :nx], want.cpu().numpy()), k
        else:
            assert_field(g[:, :nx], want.cpu().numpy(), what=("call", k))


def test_noalloc_rejects_beyond_static_buffer():
    """16384^2 with 2 * 10^5 points needs far more than the 64 MiB buffer: CGH_ENOMEM, no launch."""
    lut = cgh.wasabi_build_lut(cgh.LutParams(n_depth=64, levels=3, gamma=0.05, max_window=1024))
    q = cgh.points_tensor(200_000)
    u = torch.zeros((1, 16384), dtype=torch.complex64, device="cuda")   # row stride 16384; refused first
    rc = _noalloc(lut, q, 0, 0, 16384, 16384, u)
    assert rc == cgh.CGH_ENOMEM
    assert b"static buffer" in cgh.load().cgh_last_error()
