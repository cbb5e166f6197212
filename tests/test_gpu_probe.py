"""argus_fp64_rate and argus_mfma_rate, the device diagnostics behind the
bench's attainable rates: they run on every CU and return a plausible rate
and clock, bounded by what the units can issue at that clock."""
import math

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2510_11077_amd as A
    return A


def test_fp64_rate_is_plausible(A):
    tf1, mhz1 = A.fp64_rate(1)
    tf4, mhz4 = A.fp64_rate(4)
    print("1 wave/SIMD: %.1f TFLOP/s at %.0f MHz; 4 waves/SIMD: %.1f at %.0f" % (tf1, mhz1, tf4, mhz4))
    for tf, mhz in ((tf1, mhz1), (tf4, mhz4)):
        assert math.isfinite(tf) and math.isfinite(mhz)
        assert 300.0 < mhz < 3000.0
        # 16 FP64 FMA lanes per SIMD per cycle at the measured clock bound the rate
        assert 1.0 < tf <= 1.05 * 2 * 16 * 4 * 256 * mhz * 1e6 / 1e12


def test_fp64_rate_rejects_bad_arguments(A):
    with pytest.raises(A.ArgusError):
        A.fp64_rate(0)
    with pytest.raises(A.ArgusError):
        A.fp64_rate(5)


def test_mfma_rates_are_plausible(A):
    for kind, per_cu_cycle in ((1, 128.0), (2, 4096.0)):
        tf, mhz = A.mfma_rate(kind)
        print("MFMA kind %d: %.1f TFLOP/s at %.0f MHz" % (kind, tf, mhz))
        assert math.isfinite(tf) and 300.0 < mhz < 3000.0
        # dense FLOP per CU per clock: FP64 MFMA 128, BF16 MFMA 4096 (the
        # published 78.6 and 2,516 TFLOP/s at 2.4 GHz on 256 CUs)
        assert 1.0 < tf <= 1.05 * per_cu_cycle * 256 * mhz * 1e6 / 1e12
    with pytest.raises(A.ArgusError):
        A.mfma_rate(3)
