"""Weak-form DG on the GPU (DGX_VOL_WEAK: (2/h) sum_m Dhat_im f(u_m), the paper's other
measured solver, Section 3.1) against the oracle's weak form, element by element.

The oracle's weak form is pinned on the CPU by its identity with central flux differencing
(test_oracle_rhs.py).  Here the GPU is compared with it directly (err_v <= 1e-12) and, as a
second check independent of the oracle's weak branch, with the GPU's own central flux
differencing, which the main parity tests pin to the oracle's central branch.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_2108_06476_amd import dgx, inputs

from gpu_util import TOL_FP64, dev, err_v, host, rel_to_max

pytestmark = pytest.mark.gpu


def _cfg(dim, N, K, surface="hll", volume="weak", lo=-1.0, hi=1.0):
    cells = tuple(K) if not isinstance(K, int) else (K,) * dim
    return dict(dim=dim, polydeg=N, cells=cells, xmin=(lo,) * dim, xmax=(hi,) * dim, gamma=1.4,
                volume=volume, surface=surface)


def _state(o, kind, seed):
    if kind == "nodal":
        return inputs.random_nodal((o.E, o.NN), o.dim, seed)
    periods = [o.cfg.xmax[d] - o.cfg.xmin[d] for d in range(o.dim)]
    return inputs.random_smooth(o.node_coords(), seed, periods=periods)


def _h(cfg):
    return min((cfg["xmax"][d] - cfg["xmin"][d]) / cfg["cells"][d] for d in range(cfg["dim"]))


MATRIX = ([(3, N, "hll") for N in range(1, 8)] + [(2, N, "hll") for N in range(1, 8)] +
          [(3, 3, "llf"), (3, 3, "ec"), (3, 3, "none"), (2, 3, "llf"), (3, 4, "llf")])


@pytest.mark.parametrize("dim,N,surf", MATRIX)
@pytest.mark.parametrize("kind", ["nodal", "smooth"])
def test_weak_rhs_parity(dim, N, surf, kind):
    K = (3, 3, 2) if dim == 3 else (5, 3)          # ragged: E not a multiple of the tile
    cfg = _cfg(dim, N, K, surf)
    print("case", cfg, kind, flush=True)
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u = _state(o, kind, 200 + N)
    ref = o.rhs(u)
    got = host(s.rhs(dev(u)))
    e = err_v(got, ref, u, dim, _h(cfg))
    print("  err_v", e, "rel_to_max", rel_to_max(got, ref), flush=True)
    assert np.all(e <= TOL_FP64), e
    assert s.check() == 0


@pytest.mark.parametrize("cells", [(1, 1, 1), (1, 2, 3)])
def test_weak_thin_periodic_grids(cells):
    cfg = _cfg(3, 3, cells, "hll")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u = _state(o, "nodal", 7)
    e = err_v(host(s.rhs(dev(u))), o.rhs(u), u, 3, _h(cfg))
    assert np.all(e <= TOL_FP64), e


@pytest.mark.parametrize("N", [2, 3, 5])
def test_weak_equals_gpu_central_flux_differencing(N):
    cw = _cfg(3, N, (3, 2, 2), "hll")
    cc = _cfg(3, N, (3, 2, 2), "hll", volume="central")
    o = oracle.Oracle(**cw)
    u = _state(o, "smooth", 31)
    rw = host(dgx.Solver(**cw).rhs(dev(u)))
    rc = host(dgx.Solver(**cc).rhs(dev(u)))
    e = err_v(rw, rc, u, 3, _h(cw))
    print("weak vs central (GPU) err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e


def test_weak_full_tgv_32():
    """The full 32^3 N = 3 TGV with weak form + HLL: every element against the oracle."""
    cfg = dict(inputs.workload("tgv_32"), volume="weak", surface="hll")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u = inputs.tgv(o.node_coords())
    e = err_v(host(s.rhs(dev(u))), o.rhs(u), u, 3, 2 * np.pi / 32)
    print("weak tgv_32 err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e


def test_weak_steps_against_oracle():
    cfg = dict(inputs.scaled(inputs.workload("tgv_32"), cells=(6, 5, 4)), volume="weak",
               surface="hll")
    o = oracle.Oracle(**cfg)
    s = dgx.Solver(**cfg)
    u0 = inputs.tgv(o.node_coords())
    ref, tref = o.step(u0, 20, cfl=0.5)
    ud = dev(u0)
    t = torch.zeros(1, dtype=torch.float64, device="cuda")
    s.step(ud, 20, cfl=0.5, t=t)
    d = np.abs(host(ud) - ref).max() / np.abs(ref).max()
    print("weak 20 steps: max|du|/max|u|", d, flush=True)
    assert d <= 1e-12
    np.testing.assert_allclose(host(t)[0], tref, rtol=1e-13)


def test_weak_rejects_mixed_precision():
    with pytest.raises(dgx.DgxError):
        dgx.Solver(**dict(_cfg(3, 3, 2), precision="mixed"))


# --------------------------------------------------------------------------- matrix cores
@pytest.mark.parametrize("surf", ["hll", "llf", "ec", "none"])
@pytest.mark.parametrize("kind", ["nodal", "smooth"])
@pytest.mark.parametrize("cells", [(3, 3, 2), (1, 2, 3), (5, 1, 1)])
def test_weak_mfma_rhs_parity(surf, kind, cells):
    cfg = _cfg(3, 3, cells, surf, volume="weak_mfma")
    print("case", cfg, kind, flush=True)
    o = oracle.Oracle(**dict(cfg, volume="weak"))
    s = dgx.Solver(**cfg)
    u = _state(o, kind, 300 + cells[0])
    ref = o.rhs(u)
    got = host(s.rhs(dev(u)))
    e = err_v(got, ref, u, 3, _h(cfg))
    print("  err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e


def test_weak_mfma_full_tgv_32_and_steps():
    cfg = dict(inputs.workload("tgv_32"), volume="weak_mfma", surface="hll")
    o = oracle.Oracle(**dict(cfg, volume="weak"))
    s = dgx.Solver(**cfg)
    u = inputs.tgv(o.node_coords())
    e = err_v(host(s.rhs(dev(u))), o.rhs(u), u, 3, 2 * np.pi / 32)
    print("weak_mfma tgv_32 err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e
    small = dict(inputs.scaled(inputs.workload("tgv_32"), cells=(6, 5, 4)), volume="weak_mfma",
                 surface="hll")
    o2 = oracle.Oracle(**dict(small, volume="weak"))
    s2 = dgx.Solver(**small)
    u0 = inputs.tgv(o2.node_coords())
    ref, _ = o2.step(u0, 20, cfl=0.5)
    ud = dev(u0)
    s2.step(ud, 20, cfl=0.5)
    d = np.abs(host(ud) - ref).max() / np.abs(ref).max()
    print("weak_mfma 20 steps: max|du|/max|u|", d, flush=True)
    assert d <= 1e-12


def test_weak_mfma_matches_valu_weak():
    c = _cfg(3, 3, (4, 3, 2), "llf")
    o = oracle.Oracle(**dict(c, volume="weak"))
    u = _state(o, "smooth", 77)
    r1 = host(dgx.Solver(**c).rhs(dev(u)))
    r2 = host(dgx.Solver(**dict(c, volume="weak_mfma")).rhs(dev(u)))
    e = err_v(r2, r1, u, 3, _h(c))
    print("mfma vs valu weak err_v", e, flush=True)
    assert np.all(e <= TOL_FP64), e
