"""dgx_max_dt_noalloc (the entry point that allocates nothing: its per-element partials live
in the library's static device array) against dgx_max_dt, through the C ABI: bitwise equal
on two calls in a row, the second on a smaller state (the array keeps the first call's
values beyond the second's elements, which the second must not read), and a handle beyond
the array's 2^20 elements is rejected on the host."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2108_06476_amd import dgx, inputs

pytestmark = pytest.mark.gpu


def _pair(cells, N=3):
    cfg = inputs.scaled(inputs.workload("tgv_32"), cells=cells, polydeg=N)
    s = dgx.Solver(**cfg)
    u = inputs.tgv(s.node_coords()).contiguous()
    return s, u


@pytest.mark.parametrize("first,second", [((24, 20, 16), (6, 5, 4)), ((16, 16, 16), (3, 3, 3))])
def test_noalloc_matches_max_dt(first, second):
    for cells, cfl in ((first, 0.5), (second, 0.3)):
        print("case", cells, cfl, flush=True)
        s, u = _pair(cells)
        ref = s.max_dt(u, cfl)
        got = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        s.max_dt_noalloc(u, cfl, got)
        torch.cuda.synchronize()
        assert s.check() == 0
        assert got.item() > 0.0
        assert torch.equal(got, ref), (cells, got.item(), ref.item())


def test_noalloc_curvilinear_and_mhd_handles():
    for s, u in ((dgx.CurvSolver(3, 4), None), (dgx.MhdSolver(3, 4), None)):
        u = (inputs.mms(s.node_coords()) if isinstance(s, dgx.CurvSolver)
             else inputs.alfven(s.node_coords())).contiguous()
        ref = s.max_dt(u, 0.5)
        got = torch.zeros(1, dtype=torch.float64, device="cuda")
        s.max_dt_noalloc(u, 0.5, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref)


def test_noalloc_rejects_beyond_its_array():
    # 2D, N = 1, 1100 x 1000 elements: 1.1e6 > 2^20 (rejected before anything is enqueued)
    cfg = dict(dim=2, polydeg=1, cells=(1100, 1000), xmin=(0.0, 0.0), xmax=(1.0, 1.0),
               gamma=1.4, volume="ec", surface="llf")
    s = dgx.Solver(**cfg)
    u = torch.ones(s.shape, dtype=torch.float64, device="cuda")
    out = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    with pytest.raises(dgx.DgxError) as e:
        s.max_dt_noalloc(u, 0.5, out)
    assert "static scratch" in str(e.value)
    torch.cuda.synchronize()
    assert out.item() == 7.0
