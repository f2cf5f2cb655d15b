"""The hologram server on the GPU: every job's hologram is the same whether it runs alone (the
plain wasabi_quantize + wasabi_hologram_fused calls) or among other jobs of uneven sizes that
overlap on the device, within the FP32 tolerance; admission respects the memory budget; a small
job matches the FP64 oracle."""
import numpy as np
import pytest
import torch

import paper_1708_04233_amd as cgh
from workloads import grid_points

pytestmark = pytest.mark.gpu

TOL = 1e-5


def rel(a, b):
    return float(torch.linalg.vector_norm((a - b).flatten()) / torch.linalg.vector_norm(b.flatten()))


@pytest.fixture(scope="module")
def lut16():
    return cgh.wasabi_build_lut(cgh.LutParams(n_depth=64, levels=3, gamma=0.05, max_window=1024,
                                              value_dtype=cgh.F16))


@pytest.fixture(scope="module")
def lut_dense():
    return cgh.wasabi_build_lut(cgh.LutParams(n_depth=32, levels=3, gamma=0.6, max_window=1024))


def mix(seed, sides, counts):
    return [(side, grid_points(seed + i, n, side, side, 8, 0.1e-3, 1.5e-3))
            for i, (side, n) in enumerate(zip(sides, counts))]


def alone(lut, side, pts):
    q = cgh.wasabi_quantize(lut, torch.from_numpy(pts).cuda())
    u = cgh.wasabi_hologram_fused(lut, q, 0, 0, side, side)
    torch.cuda.synchronize()
    return u


def run_mix(lut, jobs, budget, slots):
    with cgh.Server(lut, budget, max_slots=slots) as s:
        tickets = [s.submit(p, side, side) for side, p in jobs]
        out = []
        for t, (side, p) in zip(tickets, jobs):
            r = s.wait(t, 60000)
            assert r["status"] == cgh.CGH_OK
            assert r["u"].shape == (side, side)
            out.append((r, r["u"].clone()))
            s.release(t)
        return out, s.stats()


@pytest.mark.parametrize("which", ["f16_sparse", "f32_dense"])
def test_mix_equals_alone(request, which):
    lut = request.getfixturevalue("lut16" if which == "f16_sparse" else "lut_dense")
    jobs = mix(100, [1024, 2048, 4096, 1024, 2048, 1024, 8192, 1024],
               [3000, 20000, 5000, 1000, 60000, 0, 15000, 2500])
    ref = [alone(lut, side, p) for side, p in jobs]
    out, st = run_mix(lut, jobs, 64 << 30, 2)
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["max_running"] == 2          # jobs overlapped on the device
    # results released; the slots keep their arenas and the LUT stays charged
    assert st["bytes_in_use"] == st["arena_bytes"] + st["lut_bytes"] and st["lut_bytes"] > 0
    for (r, u), want, (side, p) in zip(out, ref, jobs):
        if len(p) == 0:
            assert torch.count_nonzero(u).item() == 0
        else:
            assert rel(u, want) <= TOL, (side, len(p))
        assert r["gpu_ms"] > 0
        assert r["t_submit"] <= r["t_admit"] <= r["t_start"] <= r["t_done"]


def job_bytes(lut, side, pts):
    """Bytes the server charges for one job: its peak alone on an otherwise idle server, less the
    LUT (charged once per server)."""
    with cgh.Server(lut, 1 << 40, max_slots=1) as s:
        t = s.submit(pts, side, side)
        s.wait(t, 60000)
        st = s.stats()
        b = st["peak_bytes"] - st["lut_bytes"]
        s.release(t)
    return b


def lut_bytes(lut):
    return lut.info()["device_bytes"]


def test_tight_budget_admission(lut16):
    """Budget = the largest job's bytes: jobs that do not fit together never run together, and every
    result is still the job's hologram."""
    jobs = mix(300, [2048, 1024, 2048, 1024, 2048], [8000, 4000, 3000, 9000, 500])
    ref = [alone(lut16, side, p) for side, p in jobs]
    need = [job_bytes(lut16, side, p) for side, p in jobs]
    budget = max(need) + lut_bytes(lut16)
    out, st = run_mix(lut16, jobs, budget, 2)
    assert st["peak_bytes"] <= budget
    for i in range(len(jobs)):
        for j in range(i + 1, len(jobs)):
            if need[i] + need[j] > budget:   # j was admitted only after i's result was released
                assert out[j][0]["t_admit"] >= out[i][0]["t_done"]
    for (r, u), want in zip(out, ref):
        assert rel(u, want) <= TOL


def test_same_job_twice_in_flight(lut16):
    p = grid_points(7, 30000, 2048, 2048, 8, 0.1e-3, 1.5e-3)
    with cgh.Server(lut16, 16 << 30, max_slots=2) as s:
        a, b = s.submit(p, 2048, 2048), s.submit(p, 2048, 2048)
        ua, ub = s.wait(a, 60000)["u"].clone(), s.wait(b, 60000)["u"].clone()
        s.release(a)
        s.release(b)
    assert torch.equal(ua, ub)     # fixed-point accumulation: order-independent, bit-identical


def test_small_job_matches_oracle(orc):
    prm = orc.LutParams(n_depth=8, levels=3, gamma=0.3, max_window=1024, z_min=0.05e-3, z_max=0.2e-3)
    olut = orc.build_lut(prm)
    lut = cgh.wasabi_lut_import(cgh.LutParams(n_depth=8, levels=3, gamma=0.3, max_window=1024,
                                              z_min=0.05e-3, z_max=0.2e-3), olut.off, olut.idx, olut.val)
    nx, ny = 256, 192
    pts = grid_points(11, 300, nx, ny, 8, 0.05e-3, 0.2e-3)
    want = orc.wasabi(olut, orc.quantize(pts, prm), 0, 0, nx, ny)
    with cgh.Server(lut, 1 << 30, max_slots=2) as s:
        t = s.submit(pts, nx, ny)
        u = s.wait(t, 60000)["u"].cpu().numpy().astype(np.complex128)
        s.release(t)
    assert np.linalg.norm(u - want) / np.linalg.norm(want) <= TOL


def test_rejections_with_a_real_lut(lut16):
    with pytest.raises(cgh.CghError) as e:                       # the LUT alone fills the budget
        cgh.Server(lut16, lut_bytes(lut16), max_slots=2)
    assert e.value.code == cgh.CGH_ENOMEM
    with cgh.Server(lut16, lut_bytes(lut16) + 8 * 1024 * 1024, max_slots=2) as s:   # 8 MB: a 1024^2 result alone
        with pytest.raises(cgh.CghError) as e:
            s.submit(np.zeros((10, 4)), 1024, 1024)
        assert e.value.code == cgh.CGH_ENOMEM
        with pytest.raises(cgh.CghError) as e:
            s.submit(np.zeros((10, 4)), 100, 64)
        assert e.value.code == cgh.CGH_EINVAL


def test_forced_failure_in_a_mix(lut16):
    """One job of a mix fails while its work is issued (forced with fail_ticket, after its result
    memory was taken): it ends with CGH_EHIP, the other jobs' holograms are still each one's alone,
    and the budget gets every byte back."""
    jobs = mix(500, [1024, 2048, 1024, 2048, 1024], [3000, 8000, 2000, 6000, 4000])
    ref = [alone(lut16, side, p) for side, p in jobs]
    with cgh.Server(lut16, 16 << 30, max_slots=2, fail_ticket=3) as s:
        tickets = [s.submit(p, side, side) for side, p in jobs]
        assert tickets[2] == 3
        for k, (t, want) in enumerate(zip(tickets, ref)):
            r = s.wait(t, 60000)
            if k == 2:
                assert r["status"] == cgh.CGH_EHIP and r["u"] is None
            else:
                assert r["status"] == cgh.CGH_OK
                assert rel(r["u"].clone(), want) <= TOL
            s.release(t)
        st = s.stats()
        assert st["failed"] == 1 and st["completed"] == 4
        assert st["bytes_in_use"] == st["arena_bytes"] + st["lut_bytes"]
