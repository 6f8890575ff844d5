"""Mixed precision (float32 volume two-point fluxes and volume sums; float64 near-equal log
means, interface fluxes, lift, RK accumulation and reductions) against the float64 oracle.

The mixed path is an approximation of the float64 method, so the check is a stated error
bound, not 1e-12 parity.  Bound on the right-hand side, per field in the flux-scale norm of
gpu_util: a node sums, per direction, the volume terms S_im f#(u_i, u_m) (S = 2D - M^-1 B in
units of 2/h), each f# of size up to the flux scale and carrying a relative float32
rounding of a few units of 2^-24 from the flux algebra and the float32 accumulation; with 8
units per term the bound is 8 * 2^-24 * 3 * max_i sum_m |S_im|.  The largest absolute row
sum of S (a boundary row) grows with N: 12.2 at N = 3, 74.7 at N = 7, so the bound is
1.7e-5 and 1.1e-4.

The float32 volume sums take the pressure relative to a per-element reference (the constant
part cancels exactly against the lifted surface flux in float64): the float32 momentum terms
are then of size rho v v_d + (p - p_ref), about 1.3 at Mach 0.1 against a flux scale of
rho v v_d + p of about 72, and the momentum error stays below 1e-6 (with absolute pressures in
float32 it was 3e-6 at N = 3 and 1.4e-5 at N = 7).  The log means' float32 series branch
extends to z^2 < 1e-2 (truncation 1.1e-9), which keeps the float32 logarithm away from
b/a near 1.
"""

import numpy as np
import pytest

import oracle
from paper_2108_06476_amd import dgx, inputs

from gpu_util import dev, err_v, host, rel_to_max

pytestmark = pytest.mark.gpu



def s_rowsum(polydeg):
    """max_i sum_m |S_im|, S = 2D - M^-1 B on the LGL nodes (diagonal zero)."""
    x, w, D = oracle.lgl(polydeg)
    n = polydeg + 1
    B = np.zeros((n, n))
    B[0, 0], B[-1, -1] = -1.0, 1.0
    S = 2.0 * D - np.diag(1.0 / w) @ B
    np.fill_diagonal(S, 0.0)
    return float(np.abs(S).sum(axis=1).max())


def mixed_bound(polydeg):
    return 8 * 2.0 ** -24 * 3 * s_rowsum(polydeg)


MOMENTUM_BOUND_MACH01 = 1e-6


@pytest.mark.parametrize("name,cells", [("tgv_64_mixed", (64, 64, 64)), ("tgv_n7_32_mixed", (16, 16, 16)),
                                        ("tgv_32", (32, 32, 32))])
def test_mixed_rhs_error(name, cells):
    cfg = inputs.scaled(inputs.workload(name), cells=cells, precision="mixed")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u = inputs.tgv(o.node_coords())
    ref = o.rhs(u)
    got = host(s.rhs(dev(u)))
    h = (cfg["xmax"][0] - cfg["xmin"][0]) / cells[0]
    e = err_v(got, ref, u, 3, h)
    print(f"mixed {name} {cells}: err_v {e}  rel_to_max {rel_to_max(got, ref)}", flush=True)
    assert np.all(e <= mixed_bound(cfg["polydeg"])), e
    assert np.all(e[1:4] <= MOMENTUM_BOUND_MACH01), e   # pressure perturbation form
    assert s.check() == 0


def test_mixed_random_states():
    """Non-smooth states exercise the float32 log branch of the log means."""
    cfg = dict(dim=3, polydeg=3, cells=(3, 3, 2), xmin=(-1,) * 3, xmax=(1,) * 3, gamma=1.4,
               volume="ec", surface="llf", precision="mixed")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u = inputs.random_nodal((o.E, o.NN), 3, seed=21)
    ref = o.rhs(u)
    got = host(s.rhs(dev(u)))
    e = err_v(got, ref, u, 3, 2.0 / 3)
    print("mixed random nodal err_v", e, flush=True)
    assert np.all(e <= mixed_bound(3)), e


def test_mixed_steps_error_against_oracle():
    """50 CK(5,4) steps of the TGV on 8^3, N = 3: the state error relative to max|u| stays at
    the float32 level of the accumulated right-hand-side error (dt * steps * 5 * err)."""
    cfg = inputs.scaled(inputs.workload("tgv_32"), cells=(8, 8, 8), precision="mixed")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u0 = inputs.tgv(o.node_coords())
    ref, _ = o.step(u0, 50, cfl=0.5)
    ud = dev(u0)
    s.step(ud, 50, cfl=0.5)
    got = host(ud)
    d = np.abs(got - ref).reshape(5, -1).max(axis=1) / np.abs(ref).max()
    print("mixed 50 steps: max|du|/max|u| per field", d, flush=True)
    assert np.all(d < 1e-6), d
