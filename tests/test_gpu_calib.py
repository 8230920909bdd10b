"""The matrix-core calibration entry point (nqs_mfma_rate): a register-only
MFMA loop's sustained rate is positive and does not exceed the published
dense peaks (2.5 PFLOP/s BF16, 78.6 TFLOP/s FP64), and the two timed
launches of one configuration agree (argument checks: tests/test_abi_load.py)."""
import pytest

from paper_2204_07816_amd import nqs
from gpu_helpers import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind,peak", [("bf16", 2500.0), ("fp64", 78.6)])
def test_mfma_rate_is_below_the_published_peak(kind, peak):
    ms, tf = nqs.mfma_rate(kind, 4096, 2000 if kind == "fp64" else 8000)
    ms2, tf2 = nqs.mfma_rate(kind, 4096, 2000 if kind == "fp64" else 8000)
    say(kind, "sustained", tf, "TFLOP/s", f"{tf / peak:.1%} of the published peak", "again", tf2)
    assert 0.0 < tf <= 1.02 * peak and 0.0 < tf2 <= 1.02 * peak
    assert abs(tf - tf2) <= 0.15 * max(tf, tf2)
