"""GPU tests of continuous batching: every request's result is bit-for-bit the one it gets
when its universe's requests run alone, one after another; and each universe's chain of
windows, replayed alone one generation at a time, follows the oracle (correlation, fitness,
breeding from the warm-started population) and ends on the served result."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga, synth
from paper_1403_4099_amd.serve import GpuEngine, Request, Scheduler
from gpu_cases import fitness_tol, say

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


def test_served_window_chains_follow_the_oracle():
    """FP64 form. A short stream is served mixed; then every universe's windows are replayed
    alone in arrival order, one generation per call: the oracle correlates the same returns
    (1e-12), the first window's population is the oracle's initial population, every
    generation's fitness is within 1e-9 M of the oracle's, every next population equals the
    oracle's breed step from the GPU's population and fitness (warm starts included), and the
    replay's final best labeling and fitness equal the served ones and the oracle's choice."""
    say("serving: window chains against the oracle")
    _, stream = synth.serving_stream(duration=0.15, rate=200.0, seed=6)
    R_np = {i: R for i, (_, _, R) in enumerate(stream)}
    reqs = [Request(i, u, t, torch.from_numpy(R).cuda(), R.shape[0], R.shape[1])
            for i, (t, u, R) in enumerate(stream)]
    P, G, chunk, E = 32, 10, 5, 2
    mixed = Scheduler(GpuEngine(P=P, elites=E), P=P, generations=G, chunk=chunk, hbm_budget=4 << 30)
    res = {r.rid: r for r in mixed.run(reqs)}
    assert len(res) == len(reqs) and not mixed.rejected
    say(f"  {len(reqs)} requests served, max in flight {mixed.max_inflight}")

    eng = GpuEngine(P=P, elites=E)
    gen = {}
    for r in reqs:
        u, N = r.universe, r.N
        g0 = gen.get(u, 0)
        warm = eng.resident(u)
        inst, C, _, _ = eng.start(r, g0, warm)
        C_o = O.correlate(R_np[r.rid])
        assert float((C.cpu() - torch.from_numpy(C_o)).abs().max()) <= 1e-12, r.rid
        if warm is None:
            assert np.array_equal(inst.pop.cpu().numpy(), O.init_pop(N, P, seed=0, inst=u, gen0=0)), r.rid
        for k in range(G):
            pop_k = inst.pop.clone()
            f_k = pga.fitness(C, pop_k, "fp64").cpu().numpy()
            pop_k = pop_k.cpu().numpy()
            f_o, mag = O.fitness(C_o, pop_k, want_mag=True)
            assert np.all(np.abs(f_k - f_o) <= fitness_tol(mag)), (r.rid, k)
            eng.advance([inst], 1)
            nxt = O.breed(pop_k, f_k, E=E, seed=0, inst=u, gen=g0 + k)
            assert np.array_equal(inst.pop.cpu().numpy(), nxt), (r.rid, k)
        labels, f = eng.finish(inst)
        lab_o, f_bo, _ = O.best(inst.fitness.cpu().numpy(), inst.pop.cpu().numpy())
        assert np.array_equal(labels, lab_o) and f == f_bo, r.rid
        assert np.array_equal(labels, res[r.rid].labels) and f == res[r.rid].fitness, r.rid
        eng.keep(u, inst)
        gen[u] = g0 + G
