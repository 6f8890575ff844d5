"""The board's measured peaks (dgx_measure_peak): each within the published figure and not
implausibly far below it."""
import ctypes as C

import pytest

from paper_2108_06476_amd import dgx

pytestmark = pytest.mark.gpu


def test_measured_hbm_copy_bandwidth():
    bw = dgx.measure_peak("hbm_copy_GBs")
    print("HBM copy GB/s", bw)
    assert 2000.0 < bw < 8000.0 * 1.05


def test_measured_fp64_fma_rate():
    tf = dgx.measure_peak("fp64_fma_TFLOPs")
    print("FP64 FMA TFLOP/s", tf)
    assert 20.0 < tf < 78.6 * 1.02


def test_measure_peak_rejects_an_unknown_device():
    v = C.c_double(0.0)
    assert dgx.lib().dgx_measure_peak(4096, 0, C.byref(v)) == 1
