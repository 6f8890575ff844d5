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


@pytest.mark.parametrize("name,cells", [("tgv_32", (6, 5, 4)), ("sedov_32", (6, 5, 4)),
                                        ("tgv_32", (9, 8, 8)), ("sedov_32", (9, 8, 8)),
                                        ("density_wave_2d", None)])
def test_step_graph_equals_eager(name, cells):
    """dgx_step replays pairs of steps from its captured graph; with profiling enabled it
    launches every kernel.  Both give the same bits, over repeated calls with eager work
    between them, odd step counts, and a new state tensor (a new capture)."""
    cfg = dict(inputs.workload(name))
    if cfg["dim"] == 3:
        cfg = inputs.scaled(cfg, cells=cells)   # (9, 8, 8): above 512 elements, dt from slots
    s = dgx.Solver(**cfg)
    xyz = s.node_coords()
    if name == "tgv_32":
        u0 = inputs.tgv(xyz).contiguous()
    elif name == "sedov_32":
        u0 = torch.from_numpy(inputs.sedov(xyz.cpu().numpy())).cuda().contiguous()
    else:
        u0 = torch.from_numpy(inputs.density_wave(xyz.cpu().numpy())).cuda().contiguous()
    ug, ue = u0.clone(), u0.clone()
    tg = torch.zeros(1, dtype=torch.float64, device="cuda")
    te = torch.zeros(1, dtype=torch.float64, device="cuda")
    for n in (2, 4, 3, 2):
        s.step(ug, n, cfl=0.5, t=tg)
        _ = s.rhs(u0)                               # eager work between replays
        torch.cuda.synchronize()
        s.profile_enable(True)
        s.step(ue, n, cfl=0.5, t=te)
        s.profile_read()
        s.profile_enable(False)
        torch.cuda.synchronize()
        assert torch.equal(ug, ue), n
        assert torch.equal(tg, te), n
    u2 = u0.clone()                                 # another state tensor: recaptured
    s.step(u2, 2, cfl=0.0, dt_fixed=1e-4)
    u3 = u0.clone()
    s.profile_enable(True)
    s.step(u3, 2, cfl=0.0, dt_fixed=1e-4)
    s.profile_enable(False)
    torch.cuda.synchronize()
    assert torch.equal(u2, u3)
