"""GPU parity of the GA termination test (Algorithm 1 "determine if termination
criteria are met"; Table 3 tolerance and stall generations) against the oracle,
and its consistency properties: graph == eager, continuation, batching.

Lockstep at Table 3's tolerance: the GPU runs one generation per call; each
call is replayed by oracle_evolve_term from the GPU's population and state
(FP64 form), or checked with the oracle's termination test applied to the
GPU's own best fitness and the oracle's breed step applied to the GPU's own
fitness (both forms)."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga, synth
from gpu_cases import corr, fitness_tol, say

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _inst(C, P, G, form="fp64", **kw):
    Cg = _g(C)
    hi = lo = None
    if form == "bf16x2":
        hi, lo = pga.split(Cg)
    I = pga.make_instance(Cg, P, hi=hi, lo=lo, stats_rows=G + 1, **kw)
    I.stats.fill_(float("nan"))
    return I


def _evolve(I, G, form="fp64", init=True, eager=False, ctx=None):
    ctx = ctx or pga.Context()
    ctx.evolve([I], G, form=form, init=init, eager=eager)
    torch.cuda.synchronize()
    return I


def _same(a, b):
    return (torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness)
            and torch.equal(torch.nan_to_num(a.stats, nan=7.0), torch.nan_to_num(b.stats, nan=7.0)))


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
@pytest.mark.parametrize("k", [1, 5])
def test_huge_tolerance_stops_after_exactly_k_and_matches_oracle(form, k):
    say(f"termination k={k} {form}")
    C, _ = corr(40, seed=8)
    G = 30
    I = _evolve(_inst(C, 64, G, form, seed=9, instance_id=3, stall_gens=k, tol=1e9), G, form)
    st = I.term_state()
    assert st["stopped"] == 1 and st["gens"] == k and st["call_gens"] == k and st["stall"] == k
    s = I.stats.cpu().numpy()
    assert np.isfinite(s[: k + 1, 0]).all() and np.isnan(s[k + 1:]).all()
    if form == "fp64":
        pop_o, fit_o, st_o, state_o = O.evolve_term(C, 64, G, k, 1e9, seed=9, inst=3)
        assert np.array_equal(I.pop.cpu().numpy(), pop_o)
        assert state_o[3] == k and state_o[2] == 1
        assert np.allclose(I.fitness.cpu().numpy(), fit_o, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_stopped_run_is_the_plain_run_cut_at_the_stop(form):
    say(f"termination cut {form}")
    w = synth.config1()
    C = O.correlate(w.R)
    G = 400
    T = _evolve(_inst(C, 100, G, form, seed=0, stall_gens=20, tol=1e-5), G, form)
    st = T.term_state()
    g = st["gens"]
    assert st["stopped"] == 1 and 20 <= g < G and st["call_gens"] == g
    plain = _evolve(_inst(C, 100, g, form, seed=0), g, form)
    assert torch.equal(T.pop, plain.pop) and torch.equal(T.fitness, plain.fitness)
    assert torch.equal(T.stats[: g + 1], plain.stats)
    assert torch.isnan(T.stats[g + 1:]).all()
    # the stop is where the definition puts it, given this run's own best-fitness sequence
    best = plain.stats[:, 0].cpu().numpy()
    ref, stall, stop = -np.inf, 0, None
    for i, b in enumerate(best):
        if (np.isfinite(b) if not np.isfinite(ref) else b > ref + 1e-5 * max(1.0, abs(ref))):
            ref, stall = b, 0
        else:
            stall += 1
        if stall >= 20:
            stop = i
            break
    assert stop == g and st["ref"] == ref and st["stall"] == 20


def test_negative_tolerance_never_stops_and_equals_plain_run():
    C, _ = corr(50, seed=2)
    T = _evolve(_inst(C, 48, 15, seed=4, stall_gens=3, tol=-0.5), 15)
    P = _evolve(_inst(C, 48, 15, seed=4), 15)
    assert T.term_state()["stopped"] == 0 and T.term_state()["gens"] == 15
    assert _same(T, P)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_graph_equals_eager_and_continuation_equals_one_call(form):
    say(f"termination graph/eager/continuation {form}")
    w = synth.config1()
    C = O.correlate(w.R)
    G = 300
    a = _evolve(_inst(C, 100, G, form, seed=1, stall_gens=15, tol=1e-5), G, form)
    b = _evolve(_inst(C, 100, G, form, seed=1, stall_gens=15, tol=1e-5), G, form, eager=True)
    assert _same(a, b) and a.term_state() == b.term_state()
    g = a.term_state()["gens"]
    assert a.term_state()["stopped"] == 1 and g > 10
    # 10 generations, then continue from the state with gen0 = 10
    ctx = pga.Context()
    c = _inst(C, 100, G, form, seed=1, stall_gens=15, tol=1e-5)
    _evolve(c, 10, form, ctx=ctx)
    assert c.term_state()["gens"] == 10 and c.term_state()["stopped"] == 0
    c.gen0 = 10
    c.stats.fill_(float("nan"))
    _evolve(c, G, form, init=False, ctx=ctx)
    sa, sc = a.term_state(), c.term_state()
    assert sc["gens"] == g and sc["stopped"] == 1 and sc["call_gens"] == g - 10
    assert sa["ref"] == sc["ref"] and sa["stall"] == sc["stall"]
    assert torch.equal(a.pop, c.pop) and torch.equal(a.fitness, c.fitness)
    assert torch.equal(a.stats[10: g + 1], c.stats[: g - 10 + 1])
    # a call after the stop changes nothing and breeds nothing
    pop, fit = c.pop.clone(), c.fitness.clone()
    c.gen0 = g
    c.stats.fill_(float("nan"))
    _evolve(c, 7, form, init=False, ctx=ctx)
    assert torch.equal(c.pop, pop) and torch.equal(c.fitness, fit) and torch.isnan(c.stats).all()
    assert c.term_state()["call_gens"] == 0 and c.term_state()["gens"] == g


def test_batch_with_early_stopping_instance_equals_each_alone():
    say("termination in a ragged batch")
    specs = [  # N, P, seed, stall, tol
        (18, 100, 0, 4, 1e9),    # stops after 4 generations
        (70, 64, 1, 0, 1e-5),    # no termination test
        (130, 40, 2, 6, 1e9),    # stops after 6
        (33, 16, 3, 50, 1e-5),   # runs to the end
    ]
    G = 9
    Cs = [corr(N, seed=10 + i)[0] for i, (N, *_rest) in enumerate(specs)]
    alone = [_evolve(_inst(C, P, G, seed=s, instance_id=i, stall_gens=k, tol=t), G)
             for i, (C, (N, P, s, k, t)) in enumerate(zip(Cs, specs))]
    batch = [_inst(C, P, G, seed=s, instance_id=i, stall_gens=k, tol=t)
             for i, (C, (N, P, s, k, t)) in enumerate(zip(Cs, specs))]
    ctx = pga.Context()
    ctx.evolve(batch, G, init=True)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert _same(a, b) and a.term_state() == b.term_state()
    assert [b.term_state()["gens"] for b in batch] == [4, G, 6, G]


def _state(I):
    ts = I.term_state()
    return np.array([ts["ref"], ts["stall"], ts["stopped"], ts["gens"]], dtype=np.float64)


def _same_state(a, b):
    return (a[1:] == b[1:]).all() and (a[0] == b[0] or abs(a[0] - b[0]) <= 1e-12 * max(1.0, abs(b[0])))


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
@pytest.mark.parametrize("chunk", [1, 3, 7])
def test_any_split_into_calls_equals_one_call(form, chunk):
    """A run cut into calls of `chunk` generations is the one-call run: each generation is
    tested once, also at the call boundaries."""
    say(f"termination split into calls of {chunk} ({form})")
    w = synth.config1()
    C = O.correlate(w.R)
    G = 300
    one = _evolve(_inst(C, 60, G, form, seed=5, stall_gens=15, tol=1e-5), G, form)
    s1 = one.term_state()
    assert s1["stopped"] == 1
    ctx = pga.Context()
    I = _inst(C, 60, G, form, seed=5, stall_gens=15, tol=1e-5)
    _evolve(I, chunk, form, ctx=ctx)
    for _ in range(G):
        if I.term_state()["stopped"]:
            break
        I.gen0 = I.term_state()["gens"]
        _evolve(I, chunk, form, init=False, ctx=ctx)
    s2 = I.term_state()
    assert (s2["ref"], s2["stall"], s2["stopped"], s2["gens"]) == (s1["ref"], s1["stall"], s1["stopped"], s1["gens"])
    assert torch.equal(I.pop, one.pop) and torch.equal(I.fitness, one.fitness)


@pytest.mark.parametrize("N,P,stall,seed", [(18, 100, 20, 0), (100, 256, 12, 3)], ids=["N18-P100", "N100-P256"])
def test_lockstep_with_oracle_evolve_term_at_table3_tolerance(N, P, stall, seed):
    """FP64 form, tol 1e-5: every one-generation GPU call equals oracle_evolve_term run from the
    GPU's population and termination state (its own fitness, breeding and test), up to the stop;
    the stop generation and final population also equal the free-running oracle's."""
    say(f"termination lockstep with oracle_evolve_term N={N} P={P}")
    if N == 18:
        C = O.correlate(synth.config1().R)
    else:
        C, _ = corr(N, seed=seed)
    tol, G = 1e-5, 400
    ctx = pga.Context()
    I = _inst(C, P, G, seed=seed, instance_id=1, stall_gens=stall, tol=tol)
    state = None
    pop = None
    for g in range(G):
        if g == 0:
            _evolve(I, 1, ctx=ctx)
            pop_o, fit_o, st_o, state_o = O.evolve_term(C, P, 1, stall, tol, seed=seed, inst=1)
        else:
            I.gen0 = g
            _evolve(I, 1, init=False, ctx=ctx)
            pop_o, fit_o, st_o, state_o = O.evolve_term(C, P, 1, stall, tol, seed=seed, inst=1, pop=pop,
                                                        state=state, gen0=g)
        s_g = _state(I)
        assert _same_state(s_g, state_o), (g, s_g, state_o)
        assert np.array_equal(I.pop.cpu().numpy(), pop_o), g
        _, mag = O.fitness(C, pop_o, want_mag=True)
        assert np.all(np.abs(I.fitness.cpu().numpy() - fit_o) <= fitness_tol(mag)), g
        pop, state = I.pop.cpu().numpy(), s_g
        if s_g[2] == 1:
            break
    stop = int(state[3])
    assert state[2] == 1 and stop < G - 1
    say(f"  stopped after {stop} generations")
    pop_f, fit_f, _, state_f = O.evolve_term(C, P, G, stall, tol, seed=seed, inst=1)
    assert int(state_f[3]) == stop and state_f[2] == 1
    assert np.array_equal(pop_f, pop)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_termination_state_follows_oracle_test_on_gpu_fitness(form):
    """Both forms, tol 1e-5, generation by generation: the GPU's state after each evaluation is the
    oracle's termination test applied to the GPU's best fitness, and each new population is the
    oracle's breed step applied to the GPU's population and fitness."""
    say(f"termination state vs oracle test on GPU fitness ({form})")
    w = synth.config1()
    C = O.correlate(w.R)
    P, stall, tol, G = 100, 15, 1e-5, 400
    ctx = pga.Context()
    I = _inst(C, P, G, form, seed=2, stall_gens=stall, tol=tol)
    _evolve(I, 0, form, ctx=ctx)                     # evaluate generation 0 (a fresh state: tested)
    ref_state = O.term_test(np.array([-np.inf, 0, 0, 0.0]), float(I.fitness.max()), stall, tol)
    assert _same_state(_state(I), ref_state)
    for g in range(G):
        pop_g = I.pop.cpu().numpy()
        f_g = I.fitness.cpu().numpy()
        I.gen0 = g
        _evolve(I, 1, form, init=False, ctx=ctx)
        nxt = O.breed(pop_g, f_g, E=2, seed=2, gen=g)
        assert np.array_equal(I.pop.cpu().numpy(), nxt), g
        ref_state = O.term_test(ref_state, float(I.fitness.max()), stall, tol)
        ref_state[3] += 1.0                          # the call bred one generation
        got = _state(I)
        assert (got == ref_state).all(), (g, got, ref_state)
        if got[2] == 1:
            break
    assert ref_state[2] == 1
