"""HIP-graph capture of the per-hologram path through the entry point that allocates nothing
(wasabi_quantize + wasabi_hologram_fused_noalloc: kernel launches only, no memory nodes, no memset
nodes -- counters are cleared by the library's fill kernel).  The graph is replayed several times
with eager work and synchronisations between replays; every replay must reproduce the eager
hologram bit for bit (the binning is built from stable sorts and the sums are deterministic)."""
import pytest
import torch

import paper_1708_04233_amd as cgh
from workloads import WASABI_2048, grid_points

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("gamma", [0.84, 0.05])
def test_graph_replay_matches_eager(gamma):
    w = WASABI_2048
    lut = cgh.wasabi_build_lut(cgh.LutParams(n_depth=w["n_depth"], levels=w["levels"], gamma=gamma,
                                             max_window=w["max_window"]))
    pts = torch.from_numpy(grid_points(w["seed"], w["n"], w["nx"], w["ny"], 8, w["z_lo"], w["z_hi"])).cuda()
    q = cgh.points_tensor(pts.shape[0])
    u = torch.empty((w["ny"], w["nx"]), dtype=torch.complex64, device="cuda")

    def step():
        cgh.wasabi_quantize(lut, pts, out=q)
        cgh.wasabi_hologram_fused_noalloc(lut, q, 0, 0, w["nx"], w["ny"], u=u)

    step()
    torch.cuda.synchronize()
    eager = u.clone()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        step()                                    # warm-up on the capture stream
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        step()
    torch.cuda.synchronize()
    for k in range(4):
        u.fill_(complex(float(k), -1.0))          # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(u, eager), k


def test_allocating_entry_point_refuses_capture():
    """wasabi_hologram_fused takes its scratch from the stream-ordered pool; under capture it returns
    CGH_EINVAL before enqueueing anything (graphs holding its allocations as memory nodes are not
    supported), and the stream is usable afterwards."""
    lut = cgh.wasabi_build_lut(cgh.LutParams(n_depth=8, levels=3, gamma=0.05, max_window=256,
                                             z_min=20e-6, z_max=90e-6))
    pts = torch.from_numpy(grid_points(3, 100, 256, 256, 8, 20e-6, 90e-6)).cuda()
    q = cgh.wasabi_quantize(lut, pts)
    u = torch.empty((256, 256), dtype=torch.complex64, device="cuda")
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(cgh.CghError) as e:
        with torch.cuda.graph(g):
            cgh.wasabi_hologram_fused(lut, q, 0, 0, 256, 256, u=u)
    assert e.value.code == cgh.CGH_EINVAL and "captured" in str(e.value)
    torch.cuda.synchronize()
    want = cgh.wasabi_hologram_fused(lut, q, 0, 0, 256, 256)   # outside capture: works as before
    alone = cgh.wasabi_hologram_fused_noalloc(lut, q, 0, 0, 256, 256, u=u)
    torch.cuda.synchronize()
    assert torch.equal(alone, want)
