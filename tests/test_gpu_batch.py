"""Ensemble API (dgx_batch_*): uneven grids and polynomial degrees in one launch per RK stage
(one block per work item, or a persistent grid), steps replayed from a captured hipGraph,
autotuned or hand-set tile shape.

Each run is checked against the oracle (1e-12 in the flux-scale norm) and bitwise against
the single-run path, which computes every element with the same stage body.  Graph replays
are interleaved with eager work and synchronisations and every replay is checked.
"""

import numpy as np
import pytest
import torch

import oracle
from paper_2108_06476_amd import dgx, inputs

from gpu_util import TOL_FP64, dev, err_v, host, state_err

pytestmark = pytest.mark.gpu


def _runs(precision="fp64"):
    rng = np.random.default_rng(77)
    out = []
    for r, (N, K) in enumerate([(5, (2, 3, 2)), (3, (4, 3, 5)), (4, (3, 3, 3)), (3, (2, 2, 2)),
                                (5, (1, 2, 3)), (4, (5, 2, 1)), (3, (6, 5, 4))]):
        lo = rng.uniform(-2, 0, 3)
        hi = lo + rng.uniform(1.5, 3.0, 3)
        out.append(dict(dim=3, polydeg=N, cells=K, xmin=tuple(lo), xmax=tuple(hi),
                        gamma=float(rng.uniform(1.3, 1.67)), volume="ec",
                        surface="llf" if r % 2 == 0 else "hll", precision=precision))
    return out


def _state(o, seed):
    xyz = o.node_coords()
    periods = [o.cfg.xmax[d] - o.cfg.xmin[d] for d in range(3)]
    return inputs.random_smooth(xyz, seed, periods=periods)


def _setup(precision="fp64"):
    cfgs = _runs(precision)
    orcs = [oracle.Oracle(**c) for c in cfgs]
    us = [_state(o, 300 + r) for r, o in enumerate(orcs)]
    return cfgs, orcs, us


def test_batch_rhs_parity():
    cfgs, orcs, us = _setup()
    b = dgx.Batch(cfgs)
    ud = [dev(u) for u in us]
    dd = [torch.empty_like(u) for u in ud]
    b.rhs(ud, dd)
    for r, (c, o, u) in enumerate(zip(cfgs, orcs, us)):
        h = min((c["xmax"][d] - c["xmin"][d]) / c["cells"][d] for d in range(3))
        e = err_v(host(dd[r]), o.rhs(u), u, 3, h, c["gamma"])
        print("run", r, c["polydeg"], c["cells"], "err_v", e, flush=True)
        assert np.all(e <= TOL_FP64), (r, e)
    assert b.check() == 0


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_steps_match_single_runs_and_oracle(precision):
    cfgs, orcs, us = _setup(precision)
    b = dgx.Batch(cfgs)
    singles = [dgx.Solver(**c) for c in cfgs]
    ub = [dev(u) for u in us]
    us1 = [dev(u) for u in us]
    t = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
    for call in range(3):                       # 3 x 2 steps: one graph replay per call
        b.step(ub, 2, cfl=0.5, t=t)
        torch.cuda.synchronize()
        for s, u1 in zip(singles, us1):
            s.step(u1, 2, cfl=0.5)
        torch.cuda.synchronize()
        for r in range(len(cfgs)):
            assert torch.equal(ub[r], us1[r]), (call, r)
    assert b.check() == 0
    if precision == "fp64":
        for r, (o, u) in enumerate(zip(orcs, us)):
            ref, tref = o.step(u, 6, cfl=0.5)
            d = state_err(host(ub[r]), ref, 3)
            assert np.all(d <= 1e-12), (r, d)
            np.testing.assert_allclose(host(t)[r], tref, rtol=1e-13)


def test_batch_odd_step_counts():
    cfgs, orcs, us = _setup()
    b = dgx.Batch(cfgs)
    singles = [dgx.Solver(**c) for c in cfgs]
    ub = [dev(u) for u in us]
    us1 = [dev(u) for u in us]
    for n in (1, 3):
        b.step(ub, n, cfl=0.5)
        for s, u1 in zip(singles, us1):
            s.step(u1, n, cfl=0.5)
        torch.cuda.synchronize()
        for r in range(len(cfgs)):
            assert torch.equal(ub[r], us1[r]), (n, r)


def test_batch_tune_then_step():
    cfgs, orcs, us = _setup()
    b = dgx.Batch(cfgs)
    ub = [dev(u) for u in us]
    before = [u.clone() for u in ub]
    shape = b.tune(ub, budget_ms=500)
    print("tuned shape (threads, grid):", shape, flush=True)
    assert shape[0] in (256, 512) and shape[1] % 8 == 0
    for u0, u1 in zip(before, ub):              # tuning reads the states only
        assert torch.equal(u0, u1)
    singles = [dgx.Solver(**c) for c in cfgs]
    us1 = [u.clone() for u in ub]
    b.step(ub, 4, cfl=0.5)
    for s, u1 in zip(singles, us1):
        s.step(u1, 4, cfl=0.5)
    torch.cuda.synchronize()
    for r in range(len(cfgs)):
        assert torch.equal(ub[r], us1[r]), r


def test_batch_rejects_bad_arguments():
    cfgs, orcs, us = _setup()
    b = dgx.Batch(cfgs)
    ub = [dev(u) for u in us]
    with pytest.raises(ValueError):
        b.step(ub[:-1] + [torch.empty(3, dtype=torch.float64, device="cuda")], 1)
    bad = dict(cfgs[0], polydeg=7)
    with pytest.raises(dgx.DgxError):
        dgx.Batch([bad])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("block,grid", [(256, 16), (512, 8), (256, 40)])
def test_batch_persistent_grid(precision, block, grid):
    """A persistent grid smaller than the work-item count (every block loops over several
    items of different runs and degrees, reusing its LDS): each run bitwise equal to its
    single-run dgx_step, and (float64) within 1e-12 of the oracle after 5 steps."""
    cfgs, orcs, us = _setup(precision)
    b = dgx.Batch(cfgs)
    shape = b.set_shape(block, grid)
    print("shape (threads, grid):", shape, flush=True)
    assert shape == (block, grid)
    singles = [dgx.Solver(**c) for c in cfgs]
    ub = [dev(u) for u in us]
    us1 = [dev(u) for u in us]
    dd = [torch.empty_like(u) for u in ub]
    b.rhs(ub, dd)
    for r, (s, u1) in enumerate(zip(singles, us1)):
        assert torch.equal(dd[r], s.rhs(u1)), r
    t = torch.zeros(len(cfgs), dtype=torch.float64, device="cuda")
    for call in range(2):                       # 2 x 2 steps: graph replays of the persistent launch
        b.step(ub, 2, cfl=0.5, t=t)
        torch.cuda.synchronize()
        for s, u1 in zip(singles, us1):
            s.step(u1, 2, cfl=0.5)
        torch.cuda.synchronize()
        for r in range(len(cfgs)):
            assert torch.equal(ub[r], us1[r]), (call, r)
    b.step(ub, 1, cfl=0.5, t=t)                 # an eager (odd) step of the persistent launch
    for s, u1 in zip(singles, us1):
        s.step(u1, 1, cfl=0.5)
    torch.cuda.synchronize()
    for r in range(len(cfgs)):
        assert torch.equal(ub[r], us1[r]), ("odd", r)
    assert b.check() == 0
    if precision == "fp64":
        for r, (o, u) in enumerate(zip(orcs, us)):
            ref, tref = o.step(u, 5, cfl=0.5)
            d = state_err(host(ub[r]), ref, 3)
            print("run", r, "state err", d, flush=True)
            assert np.all(d <= 1e-12), (r, d)
            np.testing.assert_allclose(host(t)[r], tref, rtol=1e-13)


def test_batch_set_shape_rejects():
    cfgs, _, _ = _setup()
    b = dgx.Batch(cfgs)
    for block, grid in [(128, 0), (256, 12), (256, -8)]:
        with pytest.raises(dgx.DgxError):
            b.set_shape(block, grid)
    assert b.set_shape(256, 0)[0] == 256
