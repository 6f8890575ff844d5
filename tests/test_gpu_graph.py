"""The right-hand side captured in a HIP graph (as the benchmark's RHS-only line runs it):
every replay, with eager work and synchronisations between replays, equals the eager RHS
bit for bit."""
import pytest
import torch

from paper_2108_06476_amd import dgx, inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name", ["tgv_32", "sedov_32"])
def test_rhs_graph_replays_match_eager(name):
    cfg = inputs.scaled(inputs.workload(name), cells=(6, 5, 4))
    s = dgx.Solver(**cfg)
    xyz = s.node_coords()
    u = (inputs.tgv(xyz) if name == "tgv_32" else
         torch.from_numpy(inputs.sedov(xyz.cpu().numpy())).cuda()).contiguous()
    ref = s.rhs(u)
    torch.cuda.synchronize()
    du = torch.empty_like(u)
    s.rhs(u, du)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, capture_error_mode="relaxed"):
        for _ in range(3):
            s.rhs(u, du)
    for rep in range(4):
        du.zero_()
        other = s.rhs(u * 1.0001)                 # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(du, ref), rep
        del other
