"""GPU test of continuous batching: every request's result is bit-for-bit the one it gets
when its universe's requests run alone, one after another."""
import numpy as np
import pytest
import torch

from paper_1403_4099_amd import synth
from paper_1403_4099_amd.serve import GpuEngine, Request, Scheduler
from gpu_cases import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_serving_mix_equals_alone(form):
    say(f"serving mix vs alone ({form})")
    _, stream = synth.serving_stream(duration=0.5, rate=200.0, seed=4)
    reqs = [Request(i, u, t, torch.from_numpy(R).cuda(), R.shape[0], R.shape[1])
            for i, (t, u, R) in enumerate(stream)]
    P, G, chunk = 128, 20, 5
    mixed = Scheduler(GpuEngine(P=P, form=form), P=P, generations=G, chunk=chunk, hbm_budget=4 << 30, form=form)
    res = {r.rid: r for r in mixed.run(reqs)}
    assert len(res) == len(reqs) and not mixed.rejected
    assert mixed.max_inflight >= 2          # requests really overlapped on the device
    say(f"  {len(reqs)} requests, {mixed.summary()}")

    eng = GpuEngine(P=P, form=form)
    gen = {}
    for r in reqs:                          # arrival order is per-universe order
        g0 = gen.get(r.universe, 0)
        inst, C, hi, lo = eng.start(r, g0, eng.resident(r.universe))
        for _ in range(G // chunk):
            eng.advance([inst], chunk)
        labels, f = eng.finish(inst)
        eng.keep(r.universe, inst)
        gen[r.universe] = g0 + G
        assert np.array_equal(labels, res[r.rid].labels), r.rid
        assert f == res[r.rid].fitness, r.rid


def test_serving_with_termination_mix_equals_alone():
    """With the termination test on, a request retires when its GA stops; the mix still equals
    each universe's requests run alone (same stop generation, same labels and fitness)."""
    say("serving with termination, mix vs alone")
    _, stream = synth.serving_stream(duration=0.4, rate=200.0, seed=5)
    reqs = [Request(i, u, t, torch.from_numpy(R).cuda(), R.shape[0], R.shape[1])
            for i, (t, u, R) in enumerate(stream)]
    P, G, chunk, stall = 96, 60, 5, 6
    mixed = Scheduler(GpuEngine(P=P, stall_gens=stall, tol=1e-3), P=P, generations=G, chunk=chunk,
                      hbm_budget=4 << 30)
    res = {r.rid: r for r in mixed.run(reqs)}
    assert len(res) == len(reqs)
    early = [r for r in res.values() if r.gen_end % G != 0]
    say(f"  {len(reqs)} requests, {len(early)} stopped early, {mixed.summary()}")

    eng = GpuEngine(P=P, stall_gens=stall, tol=1e-3)
    gen = {}
    for r in reqs:
        g0 = gen.get(r.universe, 0)
        inst, C, hi, lo = eng.start(r, g0, eng.resident(r.universe))
        bred = 0
        for _ in range(G // chunk):
            eng.advance([inst], chunk)
            stopped, bred = eng.progress([inst])[0]
            if stopped:
                break
        labels, f = eng.finish(inst)
        eng.keep(r.universe, inst)
        gen[r.universe] = g0 + bred
        assert gen[r.universe] == res[r.rid].gen_end, r.rid
        assert np.array_equal(labels, res[r.rid].labels), r.rid
        assert f == res[r.rid].fitness, r.rid
