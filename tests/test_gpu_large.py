"""A Cartesian state beyond 2^31 values: the stage kernels' 64-bit offsets.

192^3 elements at N = 3 hold 453 M nodes, 2.26e9 values per state (the 32-bit limit is
2.15e9), 18 GB per array.  The state is a 16^3 periodic state tiled 12 times per direction
with cells of size exactly 1 on both meshes, so every element of the large mesh sees the same
data (own nodes and face neighbours) as its copy in the small one: the right-hand side and an
RK step (its dt is a maximum over the same values) must be the tiled small-mesh results bit
for bit, at every element, also those whose offsets exceed 2^31.  The small mesh is pinned
to the oracle at 1e-12.  Needs about 80 GB of device memory.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2108_06476_amd import dgx, inputs

from gpu_util import TOL_FP64, err_v, host

pytestmark = pytest.mark.gpu

KS, REP, N = 16, 12, 3


def _cfg(K):
    return dict(dim=3, polydeg=N, cells=(K, K, K), xmin=(0.0,) * 3, xmax=(float(K),) * 3,
                gamma=1.4, volume="ec", surface="llf")


def _tile(u):
    """[5][KS^3][64] -> [5][(REP KS)^3][64], element (X, Y, Z) = small element (X, Y, Z) mod KS."""
    return u.view(5, KS, KS, KS, 64).repeat(1, REP, REP, REP, 1).view(5, -1, 64)


def _equal_tiled(big, small):
    b = big.view(5, REP, KS, REP, KS, REP, KS, 64)
    s = small.view(5, 1, KS, 1, KS, 1, KS, 64)
    return bool((b == s).all().item())


def test_rhs_and_step_beyond_2_31_values():
    free, _ = torch.cuda.mem_get_info()
    if free < 100e9:
        pytest.skip(f"needs ~80 GB of free device memory, {free / 1e9:.0f} GB free")
    cs, cb = _cfg(KS), _cfg(KS * REP)
    ss = dgx.Solver(**cs)
    xyz = ss.node_coords()
    us = inputs.tgv((xyz * (2 * math.pi / KS) - math.pi).contiguous()).contiguous()
    # the small mesh against the oracle
    o = oracle.Oracle(**cs)
    ref = o.rhs(host(us))
    dus = ss.rhs(us)
    e = err_v(host(dus), ref, host(us), 3, 1.0)
    print("16^3 against the oracle: err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e

    sb = dgx.Solver(**cb)
    assert sb.nvar * sb.num_nodes > 2 ** 31
    ub = _tile(us)
    dub = sb.rhs(ub)
    torch.cuda.synchronize()
    assert _equal_tiled(dub, dus), "right-hand side of the tiled state"
    del dub
    ss.step(us, 1, cfl=0.5)
    sb.step(ub, 1, cfl=0.5)
    torch.cuda.synchronize()
    assert ss.check() == 0 and sb.check() == 0
    assert _equal_tiled(ub, us), "RK step of the tiled state"
    print(f"192^3 (N = 3): {sb.num_nodes} nodes, {sb.nvar * sb.num_nodes:.3e} values per "
          f"state: rhs and step equal the tiled 16^3 results", flush=True)
    sb.close()
    ss.close()
