"""The throughput probes (mpgemm_probe_peak) return rates in the range the
MI355X can reach: they are the measured peaks bench.py reports beside the
published ones."""
import pytest

from tests.gpu_util import note

pytestmark = pytest.mark.gpu

# (lower, upper) bounds: a tenth of and a little above the published peaks
# (FP64 78.6 TFLOP/s with FMA, 39.3 T op/s otherwise; INT8 5.0 POP/s; HBM 8 TB/s)
RANGES = {"fp64_fma": (7.86e12, 90e12), "fp64_add": (3.9e12, 45e12), "fp64_mul": (3.9e12, 45e12),
          "int8_mfma": (5e14, 5.5e15), "hbm_copy": (8e11, 8.8e12)}


@pytest.mark.parametrize("which", sorted(RANGES))
def test_probe_in_range(gpu_lib, which):
    note("probe", which)
    r = gpu_lib.probe_peak(which)
    lo, hi = RANGES[which]
    assert lo < r < hi, (which, r)


def test_probe_rejects_bad_argument(gpu_lib):
    import ctypes
    from paper_2101_06584_amd import _lib
    r = ctypes.c_double()
    assert _lib.load().mpgemm_probe_peak(7, None, ctypes.byref(r)) == -1
    assert _lib.load().mpgemm_probe_peak(-1, None, ctypes.byref(r)) == -1
    assert _lib.load().mpgemm_probe_peak(0, None, None) == -3
