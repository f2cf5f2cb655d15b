"""GPU parity of phase tables (one PSF table per depth plane and per position of a point inside its
2^L block) against the FP64 oracle, on points that are not on the 2^L grid: quantisation
(bit-exact), Eq.(2) superposition, the sub-hologram procedure and the fused tile path (relative L2
<= 1e-5, the FP32-accumulation tolerance of the other parity tests), and, with every coefficient
kept, the circ()-windowed direct sum at the points' pixel positions.

Superposition parity imports the oracle's LUT, so both sides add the same coefficients."""
import numpy as np
import pytest
import torch

import paper_1708_04233_amd as cgh
from workloads import uniform_points

pytestmark = pytest.mark.gpu
TOL = 1e-5
P = 1e-6


def _rel(u, ref):
    ref = np.asarray(ref)
    return float(np.linalg.norm((np.asarray(u, np.complex128) - ref).ravel()) /
                 max(np.linalg.norm(ref.ravel()), 1e-300))


def _kw(levels, gamma, n_depth=3, dtype=0, max_window=256):
    return dict(z_min=20e-6, z_max=90e-6, n_depth=n_depth, levels=levels, gamma=gamma,
                max_window=max_window, value_dtype=dtype, phases=1)


def _luts(orc, levels, gamma, **kw):
    k = _kw(levels, gamma, **kw)
    ref = orc.build_lut(orc.LutParams(**k))
    gpu = cgh.wasabi_lut_import(cgh.LutParams(**k), ref.off, ref.idx, ref.val)
    return ref, gpu


def _points(seed, n, nx, ny, x0, y0):
    pts = uniform_points(seed, n, nx, ny, 20e-6, 90e-6)
    pts[:, 0] += x0 * P
    pts[:, 1] += y0 * P
    return pts


def test_phase_quantize_matches_oracle(orc):
    ref, gpu = _luts(orc, 3, 0.2)
    pts = _points(4, 3000, 400, 300, -150, -120)
    pts[::97, 2] = np.nan
    pts[5, 2] = ref.params.z_max
    pts[7, :2] = [-0.5 * P, 2.5 * P]                    # ties go up: pixels (0, 3)
    q = cgh.wasabi_quantize(gpu, torch.from_numpy(pts).cuda()).cpu().numpy()
    o = orc.quantize(pts, ref.params)
    np.testing.assert_array_equal(q[:, 0], o.x)
    np.testing.assert_array_equal(q[:, 1], o.y)
    np.testing.assert_array_equal(q[:, 2], o.d)
    assert (o.d >= 0).sum() > 2000 and len(set((o.d[o.d >= 0] % 64).tolist())) == 64


@pytest.mark.parametrize("levels,gamma,sub", [(2, 0.25, 40), (3, 0.05, 64), (3, 0.6, 0),
                                              (4, 0.3, 96), (1, 0.3, 0), (3, 1.0, 64)])
def test_phase_superpose_hologram_fused_match_oracle(orc, levels, gamma, sub):
    ref, gpu = _luts(orc, levels, gamma)
    B = 1 << levels
    nx, ny, X0, Y0 = (208 // B) * B, (144 // B) * B, -B * 5, -B * 2
    pts = _points(30 + levels, 80, nx + 160, ny + 160, X0 - 80, Y0 - 80)
    q = cgh.wasabi_quantize(gpu, torch.from_numpy(pts).cuda())
    oq = orc.quantize(pts, ref.params)
    assert np.any(oq.x % B != 0)
    psi = cgh.wasabi_superpose(gpu, q, X0, Y0, nx, ny).cpu().numpy()
    assert _rel(psi, orc.superpose(ref, oq, X0, Y0, nx, ny)) < TOL
    want = orc.wasabi(ref, oq, X0, Y0, nx, ny)
    u = cgh.wasabi_hologram(gpu, q, X0, Y0, nx, ny, sub=sub).cpu().numpy()
    assert _rel(u, want) < TOL
    fused = cgh.wasabi_hologram_fused(gpu, q, X0, Y0, nx, ny).cpu().numpy()
    assert _rel(fused, want) < TOL


def test_full_phase_lut_equals_direct_sum_on_gpu(orc):
    """gamma >= 1 with phase tables: WASABI equals Eq.(1) with circ() at the points' pixels."""
    k = _kw(3, 1.0, n_depth=4)
    gpu = cgh.wasabi_build_lut(cgh.LutParams(**k))
    ref = orc.build_lut(orc.LutParams(**k))
    pts = _points(8, 200, 320, 256, -32, -32)
    q = cgh.wasabi_quantize(gpu, torch.from_numpy(pts).cuda())
    u = cgh.wasabi_hologram_fused(gpu, q, 0, 0, 256, 192).cpu().numpy()
    snapped = orc.snapped_points(orc.quantize(pts, ref.params), ref)
    d = cgh.cgh_direct(torch.from_numpy(snapped).cuda(), 256, 192, window=cgh.CIRC).cpu().numpy()
    assert _rel(u, d) < TOL
