"""Mixed precision over the full 1000-step runs of the mixed-precision workloads (N = 3 on
64^3 and N = 7 on 32^3, 16.8 M nodes each).

The float64 oracle would need about an hour per run on the host, so the reference is the
GPU float64 path, which the parity tests pin to the oracle at 1e-12 (full 32^3 right-hand
sides, steps); the oracle itself is compared with the mixed path over 50 steps in
test_gpu_mixed.py.

Bound: every right-hand-side evaluation of the mixed path is within
B = 8 * 2^-24 * 3 * max_i sum_m |S_im| of the float64 one in the flux-scale norm (the bound
of test_gpu_mixed.py), i.e.
|dR_v| <= B (2/h) F_v with F_v the largest physical flux of field v.  Five stages per step combine R with weights of order one, so after n steps of size
dt the state differs by at most about n dt B (2/h) F_v (no growth: the TGV at Mach 0.1 is
smooth over t < 0.5).  The test asserts that per field, and prints the error relative to
max|u_v|.
"""
import numpy as np
import pytest
import torch

from paper_2108_06476_amd import dgx, inputs

from gpu_util import host, phys_flux_max
from test_gpu_mixed import mixed_bound

pytestmark = pytest.mark.gpu

STEPS = 1000


@pytest.mark.parametrize("name", ["tgv_64_mixed", "tgv_n7_32_mixed"])
def test_mixed_1000_steps_against_fp64(name):
    cfg = inputs.workload(name)
    sm = dgx.Solver(**cfg)
    sd = dgx.Solver(**dict(cfg, precision="fp64"))
    u0 = inputs.tgv(sm.node_coords()).contiguous()
    um, ud = u0.clone(), u0.clone()
    tm = torch.zeros(1, dtype=torch.float64, device="cuda")
    td = torch.zeros(1, dtype=torch.float64, device="cuda")
    sm.step(um, STEPS, cfl=0.5, t=tm)
    sd.step(ud, STEPS, cfl=0.5, t=td)
    torch.cuda.synchronize()
    assert sm.check() == 0 and sd.check() == 0
    t_end = float(td.item())
    h = (cfg["xmax"][0] - cfg["xmin"][0]) / cfg["cells"][0]
    F = phys_flux_max(host(u0), 3)
    bound = t_end * mixed_bound(cfg["polydeg"]) * (2.0 / h) * F
    d = (um - ud).abs().reshape(5, -1).amax(dim=1).cpu().numpy()
    umax = ud.abs().reshape(5, -1).amax(dim=1).cpu().numpy()
    print(f"{name}: t = {t_end:.4f} after {STEPS} steps; max|du_v| {d}; bound {bound}; "
          f"relative to max|u_v| {d / umax}; t difference {float(tm.item()) - t_end:.3e}",
          flush=True)
    assert np.all(d <= bound), (d, bound)
    assert abs(float(tm.item()) - t_end) <= 1e-6 * t_end
