"""GPU parity of cgh_direct (Eq.(1)) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_1708_04233_amd as cgh
from workloads import DIRECT_512, WASABI_2048, grid_points, uniform_points

pytestmark = pytest.mark.gpu

P, LAM = 1e-6, 633e-9


def _rel(u, ref):
    return float(np.linalg.norm((u - ref).ravel()) / np.linalg.norm(ref.ravel()))


@pytest.fixture(scope="module")
def cfg512(orc):
    w = DIRECT_512
    pts = uniform_points(w["seed"], w["n"], w["nx"], w["ny"], w["z_lo"], w["z_hi"])
    ref = {win: orc.direct(pts, w["nx"], w["ny"], window=win) for win in (orc.FULL, orc.CIRC)}
    return pts, ref


@pytest.mark.parametrize("window", [cgh.FULL, cgh.CIRC])
def test_512_complex128(cfg512, window):
    pts, ref = cfg512
    u = cgh.cgh_direct(torch.from_numpy(pts).cuda(), 512, 512, window=window, out_dtype=torch.complex128)
    assert _rel(u.cpu().numpy(), ref[window]) < 1e-10


@pytest.mark.parametrize("window", [cgh.FULL, cgh.CIRC])
def test_512_complex64(cfg512, window):
    pts, ref = cfg512
    u = cgh.cgh_direct(torch.from_numpy(pts).cuda(), 512, 512, window=window, out_dtype=torch.complex64)
    got = u.cpu().numpy().astype(np.complex128)
    assert _rel(got, ref[window]) < 1e-5


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_ragged_window_offset_and_row_stride(orc, dtype):
    pts = uniform_points(3, 300, 120, 60, 20e-6, 90e-6)
    pts[:, 0] -= 30e-6   # some points left of the window
    nx, ny, ox, oy = 100, 37, -13, 7
    tol = 1e-10 if dtype == torch.complex128 else 1e-5
    for window in (cgh.FULL, cgh.CIRC):
        ref = orc.direct(pts, nx, ny, ox, oy, window=window)
        out = torch.full((ny, 128), 7.0, dtype=dtype, device="cuda")
        cgh.cgh_direct(torch.from_numpy(pts).cuda(), nx, ny, ox, oy, window=window, out=out)
        got = out.cpu().numpy()
        assert _rel(got[:, :nx].astype(np.complex128), ref) < tol
        assert np.all(got[:, nx:] == 7.0)   # padding columns untouched


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_circ_binned_path(orc, monkeypatch, dtype):
    """The tile-binned circ() path (used automatically for large problems) on a ragged window."""
    monkeypatch.setenv("CGH_DIRECT_BIN", "1")
    pts = uniform_points(9, 400, 200, 120, 20e-6, 150e-6)
    pts[:, 0] -= 40e-6
    pts[7, 2] = -1e-6                      # z <= 0 reaches nothing
    nx, ny, ox, oy = 150, 70, -17, 9
    ref = orc.direct(pts, nx, ny, ox, oy, window=orc.CIRC)
    out = torch.full((ny, 160), 2.0, dtype=dtype, device="cuda")
    cgh.cgh_direct(torch.from_numpy(pts).cuda(), nx, ny, ox, oy, window=cgh.CIRC, out=out)
    got = out.cpu().numpy()
    assert _rel(got[:, :nx].astype(np.complex128), ref) < (1e-10 if dtype == torch.complex128 else 1e-5)
    assert np.all(got[:, nx:] == 2.0)
    monkeypatch.setenv("CGH_DIRECT_BIN", "1")
    empty = cgh.cgh_direct(torch.zeros((0, 4), dtype=torch.float64, device="cuda"), 64, 32, window=cgh.CIRC)
    assert torch.count_nonzero(empty).item() == 0


def test_no_points_gives_zeros():
    pts = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    u = cgh.cgh_direct(pts, 70, 20, window=cgh.CIRC)
    assert torch.count_nonzero(u).item() == 0


def test_2048_circ_sampled_pixels(orc):
    """The 2048^2, N = 10^4 workload at full size; the oracle checks sampled 16 x 16 windows."""
    w = WASABI_2048
    pts = grid_points(w["seed"], w["n"], w["nx"], w["ny"], 8, w["z_lo"], w["z_hi"])
    u = cgh.cgh_direct(torch.from_numpy(pts).cuda(), w["nx"], w["ny"], window=cgh.CIRC).cpu().numpy()
    rng = np.random.default_rng(5)
    for _ in range(4):
        y0, x0 = (int(v) for v in rng.integers(0, w["nx"] - 16, 2))
        ref = orc.direct(pts, 16, 16, x0, y0, window=orc.CIRC)
        assert _rel(u[y0:y0 + 16, x0:x0 + 16].astype(np.complex128), ref) < 1e-5


@pytest.mark.parametrize("window", ["full", "circ"])
@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_both_tile_shapes(orc, window, dtype):
    """circ() windows of fewer than 2048 tiles of 64 x 16 pixels are summed with one row per thread
    (64 x 4 tiles), larger ones and the full window with four: each against the oracle, with a
    ragged last row of tiles."""
    win = {"full": (cgh.FULL, orc.FULL), "circ": (cgh.CIRC, orc.CIRC)}[window]
    tol = 1e-10 if dtype == torch.complex128 else 1e-5
    for nx, ny in ((2048, 1036), (200, 70)):          # 32 x 65 tiles of 64 x 16; 4 x 5
        pts = uniform_points(5, 12, nx, ny, 20e-6, 90e-6)
        u = cgh.cgh_direct(torch.from_numpy(pts).cuda(), nx, ny, window=win[0], out_dtype=dtype)
        ref = orc.direct(pts, nx, ny, window=win[1])
        assert _rel(u.cpu().numpy().astype(np.complex128), ref) < tol, (nx, ny)


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128])
def test_full_window_split_over_points(orc, dtype):
    """A small full window is summed in up to four slices of the points whose partial fields are
    added afterwards: 3000 points over a 200 x 70 window (slices of 750, not a multiple of the
    256-point batches) against the oracle."""
    nx, ny = 200, 70
    pts = uniform_points(8, 3000, nx, ny, 20e-6, 90e-6)
    u = cgh.cgh_direct(torch.from_numpy(pts).cuda(), nx, ny, window=cgh.FULL, out_dtype=dtype)
    ref = orc.direct(pts, nx, ny, window=orc.FULL)
    assert _rel(u.cpu().numpy().astype(np.complex128), ref) < (1e-10 if dtype == torch.complex128 else 1e-5)
