"""The FP64 FMA-rate probe used for the measured roofline peak: it runs, reports a plausible rate,
and rejects bad arguments before touching the device."""
import ctypes

import pytest

from paper_1808_00037_amd import teno as T

pytestmark = pytest.mark.gpu


def test_fp64_fma_probe_reports_a_plausible_rate():
    r = T.probe_fp64_fma(4096)
    # MI355X's published FP64 vector peak is 78.6 TFLOP/s; a working probe lands within a factor of 4
    assert 20.0 < r < 120.0, r


def test_fp64_fma_probe_rejects_bad_arguments():
    out = ctypes.c_double(0.0)
    assert T.lib().teno_probe_fp64_fma(None, 0, ctypes.byref(out)) == -1
    assert T.lib().teno_probe_fp64_fma(None, 1 << 25, ctypes.byref(out)) == -1
    assert T.lib().teno_probe_fp64_fma(None, 16, None) == -1
