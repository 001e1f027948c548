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


def test_pipe_mix_runs_every_mode():
    say("pipe mix loops")
    cyc = pga.pipe_mix(n_workgroups=1024, iters=1000, reps=1)
    say("  " + ", ".join(f"{k} {v:.0f}" for k, v in cyc.items()))
    assert set(cyc) == set(pga.PIPE_MIX_MODES)
    # 4 MFMAs of 16 x 16 x 32 take at least 4 x 16 cycles of the SIMD's matrix pipe (the
    # comparisons between modes are made at full size by the bench)
    assert cyc["mfma"] > 50.0
    assert all(0.0 < v < 1e5 for v in cyc.values())
