"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/dgx.h declares, and rejects invalid configurations before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_2108_06476_amd import dgx

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dgx.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dgx_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_binding_exports():
    assert sorted(dgx.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    L = C.CDLL(dgx.LIB_PATH)
    missing = [s for s in _declared() if not hasattr(L, s)]
    assert not missing, missing


@pytest.mark.parametrize("field,value", [("dim", 4), ("polydeg", 0), ("gamma", 1.0),
                                         ("volume", 9), ("surface", 7), ("precision", 5)])
def test_invalid_config_rejected_on_host(field, value):
    L = dgx.lib()
    cfg = dgx.make_config(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1))
    setattr(cfg, field, value)
    h = C.c_void_p()
    st = L.dgx_create(C.byref(cfg), None, C.byref(h))
    assert st == 1 and not h.value


@pytest.mark.parametrize("case", ["no cells", "negative cells", "empty extent", "inverted extent",
                                  "NaN gamma", "2D with cells in z", "alpha_max > 1",
                                  "alpha_min >= 1/2", "FV flux EC"])
def test_degenerate_grids_and_parameters_rejected(case):
    """Empty grids, zero-width or inverted cells and out-of-range shock-capturing parameters are
    rejected before any device call (DGX_EINVAL)."""
    L = dgx.lib()
    dim, cells, xmin, xmax = 3, [2, 2, 2], [0.0, 0.0, 0.0], [1.0, 1.0, 1.0]
    extra = {}
    if case == "no cells":
        cells[1] = 0
    elif case == "negative cells":
        cells[2] = -3
    elif case == "empty extent":
        xmax[0] = xmin[0]
    elif case == "inverted extent":
        xmax[1] = -1.0
    elif case == "NaN gamma":
        extra["gamma"] = float("nan")
    elif case == "2D with cells in z":
        dim = 2
    elif case == "alpha_max > 1":
        extra.update(volume="shockcap_hg", alpha_max=1.5)
    elif case == "alpha_min >= 1/2":
        extra.update(volume="shockcap_hg", alpha_min=0.5)
    elif case == "FV flux EC":
        extra.update(volume="shockcap_hg", fv_flux="llf")
    cfg = dgx.make_config(dim, 3, cells, xmin, xmax, **extra)
    if case == "2D with cells in z":
        cfg.cells[2] = 2
    if case == "FV flux EC":
        cfg.fv_flux = dgx.SURFACE["ec"]
    h = C.c_void_p()
    assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 1 and not h.value


def test_curved_and_mhd_parameters_rejected():
    L = dgx.lib()
    h = C.c_void_p()
    ok = dict(polydeg=3, cells=2, warp=0.1, gamma=1.4, volume=dgx.VOLUME["ec"],
              surface=dgx.SURFACE["llf"], source=0)
    for field, bad in [("cells", 0), ("warp", 0.5), ("warp", -0.1), ("polydeg", 0), ("gamma", 1.0),
                       ("surface", 9), ("source", 7)]:
        cv = dgx.CurvConfig(**dict(ok, **{field: bad}))
        assert L.dgx_create_curved(C.byref(cv), None, C.byref(h)) == 1, (field, bad)
    okm = dict(polydeg=3, cells=2, gamma=5.0 / 3.0, surface=dgx.SURFACE["hll"],
               volume=dgx.VOLUME["weak"])
    for field, bad in [("cells", 0), ("gamma", 0.9), ("volume", dgx.VOLUME["central"]),
                       ("polydeg", -1)]:
        mc = dgx.MhdConfig(**dict(okm, **{field: bad}))
        assert L.dgx_create_mhd(C.byref(mc), None, C.byref(h)) == 1, (field, bad)


def test_unsupported_config_reported():
    L = dgx.lib()
    h = C.c_void_p()
    cfg = dgx.make_config(3, 9, (2, 2, 2), (0, 0, 0), (1, 1, 1))      # polydeg not compiled
    assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 5
    cfg = dgx.make_config(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), volume="central",
                          precision="mixed")
    assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 5
    for dim, N in [(3, 4), (2, 3)]:                                   # matrix-core weak form
        cells = (2, 2, 2) if dim == 3 else (2, 2, 1)
        cfg = dgx.make_config(dim, N, cells, (0, 0, 0), (1, 1, 1), volume="weak_mfma")
        assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 5
    cfg = dgx.make_config(3, 3, (2, 2, 2), (0, 0, 0), (1, 1, 1), volume="weak", precision="mixed")
    assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 5


def test_size_limits_reported_before_any_allocation():
    """Cartesian Euler: fewer than 2^30 elements (64-bit state offsets); curvilinear and MHD
    handles: 9 (metric terms) or 8 values per node times the nodes below 2^31 (32-bit
    offsets).  The check precedes every device call."""
    L = dgx.lib()
    h = C.c_void_p()
    cfg = dgx.make_config(3, 1, (1024, 1024, 1024), (0, 0, 0), (1, 1, 1))   # 2^30 elements
    assert L.dgx_create(C.byref(cfg), None, C.byref(h)) == 5 and not h.value
    cv = dgx.CurvConfig(polydeg=3, cells=256, warp=0.1, gamma=1.4, volume=dgx.VOLUME["ec"],
                        surface=dgx.SURFACE["llf"], source=0)              # 9 * 2^30 values
    assert L.dgx_create_curved(C.byref(cv), None, C.byref(h)) == 5 and not h.value
    mc = dgx.MhdConfig(polydeg=3, cells=256, gamma=5.0 / 3.0, surface=dgx.SURFACE["hll"],
                       volume=dgx.VOLUME["weak"])                           # 8 * 2^30 values
    assert L.dgx_create_mhd(C.byref(mc), None, C.byref(h)) == 5 and not h.value


def test_null_handle_calls_fail_cleanly():
    L = dgx.lib()
    assert L.dgx_rhs(None, None, None, C.c_double(0.0)) == 1
    assert L.dgx_destroy(None) == 1
    assert L.dgx_num_nodes(None) == -1


def test_measure_peak_rejects_bad_arguments_on_host():
    """dgx_measure_peak checks its arguments before any HIP call."""
    L = dgx.lib()
    v = C.c_double(0.0)
    assert L.dgx_measure_peak(0, 0, None) == 1
    assert L.dgx_measure_peak(0, 2, C.byref(v)) == 1
    assert L.dgx_measure_peak(0, -1, C.byref(v)) == 1
