"""GPU parity of the wavelet path against the FP64 oracle: quantisation, Eq.(2) superposition,
inverse Haar transform, the sub-hologram procedure and the fused tile path.

Superposition parity uses the oracle's own LUT imported into the library, so both sides add the
same coefficients (the oracle takes no input from the GPU).  Tolerance: relative L2 <= 1e-5 for
the FP32-accumulating GPU path against the FP64 oracle, and every element within 1e-5 of the
field's peak (tests/parity.py).
"""
import numpy as np
import pytest
import torch

import paper_1708_04233_amd as cgh
from parity import assert_field
from workloads import WASABI_2048, grid_points, uniform_points

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _rel(u, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm((np.asarray(u, np.complex128) - ref).ravel()) /
                 max(np.linalg.norm(ref.ravel()), 1e-300))


def _luts(orc, levels, gamma, dtype=0, n_depth=5, z_max=90e-6, max_window=256):
    kw = dict(z_min=20e-6, z_max=z_max, n_depth=n_depth, levels=levels, gamma=gamma,
              max_window=max_window, value_dtype=dtype)
    ref = orc.build_lut(orc.LutParams(**kw))
    gpu = cgh.wasabi_lut_import(cgh.LutParams(**kw), ref.off, ref.idx, ref.val)
    return ref, gpu


def _points(seed, n, nx, ny, B, x0=0, y0=0, z=(20e-6, 90e-6)):
    return grid_points(seed, n, nx, ny, B, z[0], z[1], x0=x0, y0=y0)


def _q_gpu(gpu_lut, pts):
    return cgh.wasabi_quantize(gpu_lut, torch.from_numpy(pts).cuda())


def test_quantize_matches_oracle(orc):
    ref, gpu = _luts(orc, 3, 0.2)
    pts = uniform_points(4, 2000, 400, 300, 10e-6, 100e-6)
    pts[:, :2] -= 150e-6                      # negative coordinates
    pts[::97, 2] = np.nan                     # non-finite -> invalid
    pts[5, 2] = ref.params.z_max              # top plane edge
    pts[6, 2] = ref.params.z_min
    q = _q_gpu(gpu, pts).cpu().numpy()
    o = orc.quantize(pts, ref.params)
    np.testing.assert_array_equal(q[:, 0], o.x)
    np.testing.assert_array_equal(q[:, 1], o.y)
    np.testing.assert_array_equal(q[:, 2], o.d)
    np.testing.assert_array_equal(q[:, 3].view(np.float32), o.a.astype(np.float32))
    assert (o.d == -1).sum() > 100 and (o.d >= 0).sum() > 100


# gamma < 0.35 runs the sparse (value, key) path, gamma >= 0.35 the dense-block path
CASES = [(1, 0.3, 0), (2, 0.2, 0), (3, 0.05, 0), (3, 0.6, 0), (4, 0.3, 0), (5, 0.3, 0),
         (6, 0.5, 0), (3, 0.3, 1), (3, 0.3, 2), (1, 0.6, 0), (2, 0.5, 0), (4, 0.9, 0),
         (3, 0.84, 1), (3, 0.84, 2), (5, 1.0, 0)]


@pytest.mark.parametrize("levels,gamma,dtype", CASES)
def test_superpose_matches_oracle(orc, levels, gamma, dtype):
    ref, gpu = _luts(orc, levels, gamma, dtype)
    B = 1 << levels
    # ragged window (not a multiple of the 64-pixel tile unless B = 64), negative origin
    nx, ny = (200 // B) * B if B < 64 else 192, (136 // B) * B if B < 64 else 128
    X0, Y0 = -B * 2, B * 3
    pts = _points(10 + levels, 60, nx + 160, ny + 160, B, x0=X0 - 80, y0=Y0 - 80)
    q = _q_gpu(gpu, pts)
    psi = cgh.wasabi_superpose(gpu, q, X0, Y0, nx, ny).cpu().numpy()
    want = orc.superpose(ref, orc.quantize(pts, ref.params), X0, Y0, nx, ny)
    assert_field(psi, want)


@pytest.mark.parametrize("levels,nx", [(3, 200), (4, 208), (3, 64)])
def test_superpose_into_unaligned_field(orc, levels, nx):
    """The Mallat field written 8 bytes past a 16-byte boundary (coefficients stored one at a time
    instead of two per store): bitwise the same as into an aligned field (fixed-point sums), and
    equal to the oracle.  nx = 208 at L = 4 gives an odd scaling-band width (13)."""
    ref, gpu = _luts(orc, levels, 0.25)
    B = 1 << levels
    ny = 136 // B * B
    X0, Y0 = -B * 3, B
    pts = _points(40 + levels, 60, nx + 160, ny + 160, B, x0=X0 - 80, y0=Y0 - 80)
    q = _q_gpu(gpu, pts)
    aligned = cgh.wasabi_superpose(gpu, q, X0, Y0, nx, ny)
    flat = torch.full((nx * ny + 1,), complex("nan"), dtype=torch.complex64, device="cuda")
    view = flat[1:].view(ny, nx)
    assert view.data_ptr() % 16 == 8
    cgh.wasabi_superpose(gpu, q, X0, Y0, nx, ny, psi=view)
    torch.cuda.synchronize()
    assert torch.equal(aligned, view)
    assert torch.isnan(flat[0])                    # nothing written before the field
    want = orc.superpose(ref, orc.quantize(pts, ref.params), X0, Y0, nx, ny)
    assert_field(aligned.cpu().numpy(), want)


@pytest.mark.parametrize("levels", [1, 2, 3, 4, 5, 6])
def test_idwt_matches_oracle(orc, levels):
    B = 1 << levels
    nx, ny = max(B, (200 // B) * B), max(B, (72 // B) * B)
    rng = np.random.default_rng(levels)
    psi = (rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))).astype(np.complex64)
    u = torch.full((ny, nx + 24), 3.0, dtype=torch.complex64, device="cuda")
    cgh.wasabi_idwt(torch.from_numpy(psi).cuda(), levels, u=u)
    got = u.cpu().numpy()
    assert_field(got[:, :nx], orc.haar_inverse(psi.astype(np.complex128), levels), tol=1e-6, elem=1e-6)
    assert np.all(got[:, nx:] == 3.0)


@pytest.mark.parametrize("levels,sub,gamma", [(3, 64, 0.25), (3, 0, 0.25), (4, 96, 0.25),
                                              (2, 40, 0.25), (3, 64, 0.84), (4, 96, 0.6),
                                              (1, 0, 0.25), (5, 0, 0.25), (6, 0, 0.25)])
def test_hologram_and_fused_match_oracle(orc, levels, sub, gamma):
    ref, gpu = _luts(orc, levels, gamma)
    B = 1 << levels
    nx, ny, X0, Y0 = (208 // B) * B, (144 // B) * B, -B * 5, -B * 2
    pts = _points(30 + levels, 80, nx + 160, ny + 160, B, x0=X0 - 80, y0=Y0 - 80)
    q = _q_gpu(gpu, pts)
    want = orc.wasabi(ref, orc.quantize(pts, ref.params), X0, Y0, nx, ny)
    u = torch.full((ny, nx + 8), 5.0, dtype=torch.complex64, device="cuda")
    cgh.wasabi_hologram(gpu, q, X0, Y0, nx, ny, sub=sub, u=u)
    got = u.cpu().numpy()
    assert_field(got[:, :nx], want)
    assert np.all(got[:, nx:] == 5.0)
    fused = cgh.wasabi_hologram_fused(gpu, q, X0, Y0, nx, ny).cpu().numpy()
    assert_field(fused, want)
    # into a view whose rows are not 16-byte aligned (odd row stride, 8-byte offset)
    big = torch.full((ny, nx + 9), 7.0, dtype=torch.complex64, device="cuda")
    view = big[:, 1:1 + nx]
    cgh.wasabi_hologram_fused(gpu, q, X0, Y0, nx, ny, u=view)
    got = big.cpu().numpy()
    assert_field(got[:, 1:1 + nx], want)
    # sparse: fixed-point sums; dense: FP32 sums in the order of lists built by stable sorts --
    # bitwise the same as the aligned output either way
    assert np.array_equal(got[:, 1:1 + nx], fused)
    assert np.all(got[:, 0] == 7.0) and np.all(got[:, 1 + nx:] == 7.0)


def test_no_points_and_invalid_points(orc):
    ref, gpu = _luts(orc, 3, 0.3)
    q = cgh.points_tensor(0)
    assert torch.count_nonzero(cgh.wasabi_hologram_fused(gpu, q, 0, 0, 72, 64)).item() == 0
    assert torch.count_nonzero(cgh.wasabi_superpose(gpu, q, 0, 0, 72, 64)).item() == 0
    pts = _points(2, 50, 64, 64, 8)
    pts[:, 2] = 1.0                           # every point beyond z_max -> invalid
    q = _q_gpu(gpu, pts)
    assert torch.count_nonzero(cgh.wasabi_hologram(gpu, q, 0, 0, 64, 64)).item() == 0


def test_window_argument_checks(orc):
    ref, gpu = _luts(orc, 3, 0.3)
    q = cgh.points_tensor(4)
    for bad in [(4, 0, 64, 64), (0, 0, 60, 64), (0, 0, 64, 0)]:
        with pytest.raises(cgh.CghError):
            cgh.wasabi_superpose(gpu, q, *bad, psi=torch.empty((bad[3], bad[2]),
                                                                  dtype=torch.complex64, device="cuda"))
    with pytest.raises(cgh.CghError):
        cgh.wasabi_hologram(gpu, q, 0, 0, 64, 64, sub=12)


def test_full_lut_equals_direct_sum_on_gpu(orc):
    """gamma >= 1 with on-grid points: WASABI equals the circ()-windowed Eq.(1) sum."""
    kw = dict(z_min=20e-6, z_max=90e-6, n_depth=6, levels=3, gamma=1.0, max_window=256)
    gpu = cgh.wasabi_build_lut(cgh.LutParams(**kw))
    pts = _points(8, 200, 320, 256, 8, x0=-32, y0=-32)
    q = _q_gpu(gpu, pts)
    u = cgh.wasabi_hologram_fused(gpu, q, 0, 0, 256, 192).cpu().numpy()
    snapped = orc.snapped_points(orc.quantize(pts, orc.LutParams(**kw)), orc.build_lut(orc.LutParams(**kw)))
    d = cgh.cgh_direct(torch.from_numpy(snapped).cuda(), 256, 192, window=cgh.CIRC).cpu().numpy()
    assert_field(u, d)


def test_own_lut_end_to_end(orc):
    """GPU-built LUT end to end against the oracle-built LUT (the same selection rule)."""
    kw = dict(z_min=20e-6, z_max=90e-6, n_depth=6, levels=3, gamma=0.2, max_window=256)
    gpu = cgh.wasabi_build_lut(cgh.LutParams(**kw))
    ref = orc.build_lut(orc.LutParams(**kw))
    pts = _points(9, 150, 320, 256, 8, x0=-32, y0=-32)
    u = cgh.wasabi_hologram_fused(gpu, _q_gpu(gpu, pts), 0, 0, 256, 192).cpu().numpy()
    want = orc.wasabi(ref, orc.quantize(pts, ref.params), 0, 0, 256, 192)
    assert_field(u, want)


def test_2048_workload_sampled_windows(orc):
    """The 2048^2, N = 10^4, 64-plane, L = 3, gamma = 5% workload at full size (oracle LUT
    imported); the oracle computes four 128 x 128 windows (Haar windows are exact)."""
    w = WASABI_2048
    kw = dict(n_depth=w["n_depth"], levels=w["levels"], gamma=w["gamma"], max_window=w["max_window"])
    ref = orc.build_lut(orc.LutParams(**kw))
    gpu = cgh.wasabi_lut_import(cgh.LutParams(**kw), ref.off, ref.idx, ref.val)
    pts = grid_points(w["seed"], w["n"], w["nx"], w["ny"], 8, w["z_lo"], w["z_hi"])
    q = _q_gpu(gpu, pts)
    full = cgh.wasabi_hologram_fused(gpu, q, 0, 0, w["nx"], w["ny"]).cpu().numpy()
    split = cgh.wasabi_hologram(gpu, q, 0, 0, w["nx"], w["ny"], sub=1024).cpu().numpy()
    oq = orc.quantize(pts, ref.params)
    rng = np.random.default_rng(11)
    for k in range(4):
        y0, x0 = (int(v) * 8 for v in rng.integers(0, (w["nx"] - 128) // 8, 2))
        want = orc.wasabi(ref, oq, x0, y0, 128, 128)
        assert_field(full[y0:y0 + 128, x0:x0 + 128], want, what=(k, x0, y0))
        assert_field(split[y0:y0 + 128, x0:x0 + 128], want, what=(k, x0, y0))


@pytest.mark.parametrize("levels,gamma", [(3, 0.25), (3, 0.84), (4, 0.3), (4, 0.6)])
def test_superpose_accumulate(orc, levels, gamma):
    """accumulate = 1 adds the call's field to psi: the field of a point set superposed in two
    halves (overwrite, then add) equals the oracle's field of all points, for the sparse
    (gamma < 0.35) and the dense kernel."""
    ref, gpu = _luts(orc, levels, gamma)
    B = 1 << levels
    nx, ny, X0, Y0 = (200 // B) * B, (136 // B) * B, -B * 2, B * 3
    pts = _points(50 + levels, 90, nx + 160, ny + 160, B, x0=X0 - 80, y0=Y0 - 80)
    q = _q_gpu(gpu, pts)
    half = q.shape[0] // 2
    psi = torch.full((ny, nx), complex(9.0, -9.0), dtype=torch.complex64, device="cuda")
    cgh.wasabi_superpose(gpu, q[:half].contiguous(), X0, Y0, nx, ny, psi=psi)
    first = psi.clone()
    cgh.wasabi_superpose(gpu, q[half:].contiguous(), X0, Y0, nx, ny, psi=psi, accumulate=True)
    oq = orc.quantize(pts, ref.params)
    want_first = orc.superpose(ref, orc.quantize(pts[:half], ref.params), X0, Y0, nx, ny)
    assert_field(first.cpu().numpy(), want_first, what="first half, overwritten")
    assert_field(psi.cpu().numpy(), orc.superpose(ref, oq, X0, Y0, nx, ny), what="both halves")
    # the inverse of the accumulated field is the hologram of all points
    u = cgh.wasabi_idwt(psi, levels).cpu().numpy()
    assert_field(u, orc.wasabi(ref, oq, X0, Y0, nx, ny), what="hologram")


@pytest.mark.parametrize("levels", [1, 3, 4, 6])
def test_idwt_in_place(orc, levels):
    """u == psi: the field is replaced by its inverse (the library inverts a copy)."""
    B = 1 << levels
    nx, ny = max(B, (200 // B) * B), max(B, (136 // B) * B)
    rng = np.random.default_rng(100 + levels)
    psi = (rng.normal(size=(ny, nx)) + 1j * rng.normal(size=(ny, nx))).astype(np.complex64)
    field = torch.from_numpy(psi).cuda()
    out = cgh.wasabi_idwt(field, levels, u=field)
    assert out.data_ptr() == field.data_ptr()
    assert_field(field.cpu().numpy(), orc.haar_inverse(psi.astype(np.complex128), levels), tol=1e-6, elem=1e-6)
    # u one row further into the same memory overlaps psi only partly: refused
    flat = torch.zeros(nx * ny + nx, dtype=torch.complex64, device="cuda")
    with pytest.raises(cgh.CghError) as e:
        cgh.wasabi_idwt(flat[:nx * ny].view(ny, nx), levels, u=flat[nx:].view(ny, nx))
    assert e.value.code == cgh.CGH_EINVAL


@pytest.mark.parametrize("gamma,side,n", [(0.84, 2048, 10_000), (0.05, 2048, 10_000), (0.6, 8192, 20_000),
                                         (0.2, 8192, 20_000)])
def test_repeated_runs_bitwise(gamma, side, n):
    """The same input run several times in one process gives the same hologram bit for bit.  The
    2048^2 grid takes the chunk-matrix lists and plane pacing, 8192^2 (16384 tiles) the lists per
    2 x 2 tile cell; gamma >= 0.35 runs the dense kernel (FP32 sums in list order), gamma < 0.35 the
    sparse one (fixed-point sums).  The plane sort and the list builds are stable sorts, so the
    dense kernel's FP32 sums run in the same order every time."""
    lut = cgh.wasabi_build_lut(cgh.LutParams(n_depth=64, levels=3, gamma=gamma, max_window=1024))
    pts = grid_points(70, n, side, side, 8, 0.1e-3, 1.5e-3)
    q = cgh.wasabi_quantize(lut, torch.from_numpy(pts).cuda())
    nan = complex(float("nan"), float("nan"))
    first = cgh.wasabi_hologram_fused(lut, q, 0, 0, side, side,
                                      u=torch.full((side, side), nan, dtype=torch.complex64, device="cuda")).clone()
    assert bool(torch.isfinite(torch.view_as_real(first)).all())   # every tile written
    for _ in range(3):
        again = cgh.wasabi_hologram_fused(lut, q, 0, 0, side, side)
        torch.cuda.synchronize()
        assert torch.equal(again, first)
    psi0 = cgh.wasabi_superpose(lut, q, 0, 0, side, side).clone()
    psi1 = cgh.wasabi_superpose(lut, q, 0, 0, side, side)
    torch.cuda.synchronize()
    assert torch.equal(psi0, psi1)
    # the separate path (psi, then the inverse, whose tiles go in row-major order) gives the same bits
    assert torch.equal(cgh.wasabi_idwt(psi0, 3), first)
