"""GPU check of the measurement aid behind the bench's measured MFMA ceiling: it runs, its sink
values are finite, and the rate it reports is a plausible fraction of the published peak."""
import pytest

from paper_1403_4099_amd import pga
from gpu_cases import say

pytestmark = pytest.mark.gpu


def test_peak_mfma_bf16_rate_is_plausible():
    say("peak MFMA bf16 loop")
    tf = pga.peak_mfma_bf16(n_workgroups=1024, iters=200, reps=3)
    say(f"  {tf:.0f} TFLOP/s")
    assert 100.0 < tf < 2600.0     # published dense peak 2500 TFLOP/s; rounding slack above


def test_peak_fp64_rate_is_plausible():
    say("peak FP64 FMA loop")
    tf = pga.peak_fp64(n_workgroups=1024, iters=400, reps=3)
    say(f"  {tf:.1f} TFLOP/s")
    assert 5.0 < tf < 82.0         # published FP64 vector peak 78.6 TFLOP/s; rounding slack above
