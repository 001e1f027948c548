"""GPU parity of the GA (init, rank/stats, breed, evolve, best) against the CPU oracle.

Lockstep protocol: the GPU's population at generation g and the GPU fitness
of it are handed to the oracle's breed step, whose output must equal the
GPU's next population bit for bit; the GPU fitness itself is checked against
the oracle's within the FP64 tolerance.
"""
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
    return pga.make_instance(Cg, P, hi=hi, lo=lo, stats_rows=G + 1, **kw)


@pytest.mark.parametrize("N,P,seed,inst,gen0", [(18, 100, 0, 0, 0), (37, 50, 7, 5, 11), (300, 70, 2**40 + 3, 9, 2**31)])
def test_init_population_bit_exact(N, P, seed, inst, gen0):
    say(f"init N={N} P={P}")
    C, _ = corr(N, seed=1)
    ctx = pga.Context()
    I = _inst(C, P, 0, seed=seed, instance_id=inst, gen0=gen0)
    ctx.evolve([I], 0, init=True)
    pop = I.pop.cpu().numpy()
    assert np.array_equal(pop, O.init_pop(N, P, seed=seed, inst=inst, gen0=gen0))
    f_o, mag = O.fitness(C, pop, want_mag=True)
    assert np.all(np.abs(I.fitness.cpu().numpy() - f_o) <= fitness_tol(mag))
    st = I.stats.cpu().numpy()[0]
    so = O.stats(I.fitness.cpu().numpy())
    assert st[0] == so[0] and st[2] == so[2] and st[3] == so[3]
    assert st[1] == pytest.approx(so[1], rel=1e-12)


LOCK_CASES = [
    # N, P, E, generations, form
    (18, 100, 2, 12, "fp64"),
    (37, 50, 3, 6, "fp64"),
    (130, 64, 0, 4, "fp64"),
    (300, 40, 5, 3, "fp64"),
    (18, 100, 2, 6, "bf16x2"),
    (257, 48, 2, 3, "bf16x2"),
    (516, 40, 1, 3, "bf16x2"),     # several 128-gene crossover blocks per child
    (1028, 24, 2, 2, "fp64"),      # more gene pairs than threads: a second round
]


@pytest.mark.parametrize("N,P,E,G,form", LOCK_CASES, ids=[f"N{c[0]}-P{c[1]}-E{c[2]}-{c[4]}" for c in LOCK_CASES])
def test_breed_lockstep_with_oracle(N, P, E, G, form):
    say(f"lockstep N={N} P={P} E={E} {form}")
    C, _ = corr(N, seed=3)
    ctx = pga.Context()
    I = _inst(C, P, 1, form=form, elites=E, seed=77, instance_id=2)
    ctx.evolve([I], 0, form=form, init=True)
    for g in range(G):
        pop_g = I.pop.clone()
        f_g = pga.fitness(I.C, pop_g, form, hi=I.hi, lo=I.lo)
        assert torch.equal(f_g, I.fitness)                      # evolve's fitness == pga_fitness, bitwise
        if form == "fp64":
            f_o, mag = O.fitness(C, pop_g.cpu().numpy(), want_mag=True)
            assert np.all(np.abs(f_g.cpu().numpy() - f_o) <= fitness_tol(mag))
        I.gen0 = g
        ctx.evolve([I], 1, form=form, eager=(g % 2 == 0))
        nxt = O.breed(pop_g.cpu().numpy(), f_g.cpu().numpy(), E=E, seed=77, inst=2, gen=g)
        assert np.array_equal(I.pop.cpu().numpy(), nxt), f"generation {g}"
        st = I.stats.cpu().numpy()
        so = O.stats(f_g.cpu().numpy())
        assert st[0, 0] == so[0] and st[0, 2] == so[2] and st[0, 3] == so[3]


def _run(C, P, G, form, eager, seed=5, inst=0, pop=None, gen0=0, E=2):
    ctx = pga.Context()
    I = _inst(C, P, G, form=form, elites=E, seed=seed, instance_id=inst, gen0=gen0,
              pop=None if pop is None else pop.clone())
    ctx.evolve([I], G, form=form, init=pop is None, eager=eager)
    torch.cuda.synchronize()
    return I


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_graph_equals_eager_and_resume_is_exact(form):
    say(f"graph/eager/resume {form}")
    C, _ = corr(64, seed=4)
    a = _run(C, 80, 9, form, eager=False)
    b = _run(C, 80, 9, form, eager=True)
    assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness) and torch.equal(a.stats, b.stats)
    # replaying the cached graph again gives the same result
    ctx = pga.Context()
    c = _inst(C, 80, 9, form=form, seed=5)
    for _ in range(2):
        ctx.evolve([c], 9, form=form, init=True)
        assert torch.equal(a.pop, c.pop) and torch.equal(a.fitness, c.fitness)
    # 0 -> 4 then 4 -> 9 equals 0 -> 9
    h = _run(C, 80, 4, form, eager=False)
    r = _run(C, 80, 5, form, eager=False, pop=h.pop, gen0=4)
    assert torch.equal(a.pop, r.pop) and torch.equal(a.fitness, r.fitness)
    assert torch.equal(a.stats[4:], r.stats)


def test_batched_instances_equal_each_alone():
    say("batched == alone")
    specs = [(18, 100, 0, 11), (70, 64, 1, 12), (130, 40, 2, 13), (33, 10, 3, 14)]
    G = 7
    alone = []
    for N, P, iid, seed in specs:
        C, _ = corr(N, seed=iid)
        alone.append(_run(C, P, G, "fp64", eager=False, seed=seed, inst=iid, E=1 + iid % 3))
    ctx = pga.Context()
    insts = []
    for (N, P, iid, seed) in specs:
        C, _ = corr(N, seed=iid)
        insts.append(_inst(C, P, G, elites=1 + iid % 3, seed=seed, instance_id=iid))
    ctx.evolve(insts, G, init=True)
    torch.cuda.synchronize()
    for a, b in zip(alone, insts):
        assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness) and torch.equal(a.stats, b.stats)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_ragged_batch_of_batched_workload_instances_equals_alone(form):
    """24 instances of the batched workload (N ~ U{32..512}) in one evolve call == each alone."""
    say(f"ragged batch of 24 ({form})")
    G, P = 4, 64
    ws = [synth.config4_instance(i, T=128) for i in range(24)]
    Cs = [O.correlate(w.R) for w in ws]
    alone = [_run(C, P, G, form, eager=False, seed=3, inst=i) for i, C in enumerate(Cs)]
    ctx = pga.Context()
    insts = [_inst(C, P, G, form=form, seed=3, instance_id=i) for i, C in enumerate(Cs)]
    ctx.evolve(insts, G, form=form, init=True)
    torch.cuda.synchronize()
    for a, b in zip(alone, insts):
        assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness) and torch.equal(a.stats, b.stats)
    if form == "fp64":
        for C, b in zip(Cs, insts):
            f_o, mag = O.fitness(C, b.pop.cpu().numpy(), want_mag=True)
            assert np.all(np.abs(b.fitness.cpu().numpy() - f_o) <= fitness_tol(mag))


def test_free_running_config1_recovers_planted_and_matches_oracle():
    say("free-running config 1")
    w = synth.config1()
    C = O.correlate(w.R)
    I = _run(C, w.P, w.G, "fp64", eager=False, seed=w.seed, E=w.elites)
    lab, f, idx = pga.best(I.fitness, I.pop)
    assert np.array_equal(lab, O.canonical(w.planted))
    pop_o, fit_o, st_o = O.evolve(C, P=w.P, G=w.G, E=w.elites, seed=w.seed)
    lab_o, f_o, _ = O.best(fit_o, pop_o)
    assert np.array_equal(lab, lab_o)
    assert f == pytest.approx(f_o, rel=1e-12)
    st = I.stats.cpu().numpy()
    assert np.all(np.diff(st[:, 0]) >= 0.0)
    first_diff = next((g for g in range(w.G + 1) if st[g, 3] != st_o[g, 3]), None)
    say(f"  first generation whose argbest differs from the free-running oracle: {first_diff}")


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_best_matches_oracle(form):
    C, _ = corr(100, seed=6)
    I = _run(C, 64, 5, form, eager=False)
    lab, f, idx = pga.best(I.fitness, I.pop)
    lab_o, f_o, idx_o = O.best(I.fitness.cpu().numpy(), I.pop.cpu().numpy())
    assert np.array_equal(lab, lab_o) and f == f_o and idx == idx_o


def test_best_with_ties_and_invalid():
    f = _g(np.array([-np.inf, 3.0, 3.0, 1.0]))
    pop = _g(np.array([[0, 0, 0], [2, 1, 2], [0, 1, 2], [1, 1, 1]], dtype=np.int32))
    lab, fb, idx = pga.best(f, pop)
    assert idx == 1 and fb == 3.0 and list(lab) == [0, 1, 0]


def test_capacity_sized_graph_serves_mixes_that_round_alike():
    """pga_evolve rounds its launch sizes up (four values per octave) and pads the instance list:
    a mix whose sizes round to the same values replays the cached graph, padding workgroups and
    slots do nothing, and every result equals its eager run bit for bit."""
    say("capacity-sized graph reuse")
    G = 3
    mixes = [[(70, 64, 0), (130, 40, 1), (33, 10, 2)],       # 114 individuals -> launch size 128
             [(71, 64, 3), (129, 40, 4), (35, 12, 5)]]       # 116 individuals -> 128 as well
    ctx = pga.Context()
    ctx.ws = torch.empty(64 << 20, dtype=torch.uint8, device=DEV)   # one workspace: one graph key
    for form in ("fp64", "bf16x2"):
        for mix in mixes:
            Cs = [corr(N, seed=iid)[0] for N, P, iid in mix]
            eager = [_inst(C, P, G, form=form, seed=9, instance_id=iid) for C, (N, P, iid) in zip(Cs, mix)]
            pga.Context().evolve(eager, G, form=form, init=True, eager=True)
            graph = [_inst(C, P, G, form=form, seed=9, instance_id=iid) for C, (N, P, iid) in zip(Cs, mix)]
            ctx.evolve(graph, G, form=form, init=True)
            torch.cuda.synchronize()
            for a, b in zip(eager, graph):
                assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness)
                assert torch.equal(a.stats, b.stats)
        assert ctx.graphs() == (1 if form == "fp64" else 2)


@pytest.mark.parametrize("N,P,E", [(40, 600, 2), (300, 96, 4), (300, 96, 6), (1100, 80, 3), (1100, 80, 0)],
                         ids=["N40-E2", "N300-E4", "N300-E6", "N1100-E3", "N1100-E0"])
def test_breed_ranking_paths_agree_bitwise(N, P, E):
    # Without SUS or an early stop the breed launch ranks each instance itself;
    # an armed termination test that never fires runs the rank kernel first.
    # Both must give the same populations, fitnesses and statistics bits, for
    # the wave-per-slot (N <= 1024) and workgroup-per-slot breed, with elites
    # within and beyond what a single read of the fitnesses ranks.
    say(f"ranking paths N={N} P={P} E={E}")
    C, _ = corr(N, seed=8)
    G = 5
    runs = []
    for stall in (0, 10**6):
        I = _inst(C, P, G, form="fp64", elites=E, seed=13, instance_id=1, stall_gens=stall, tol=1e300)
        pga.Context().evolve([I], G, form="fp64", init=True)
        torch.cuda.synchronize()
        runs.append(I)
    a, b = runs
    assert b.term_state()["stopped"] == 0
    assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness) and torch.equal(a.stats, b.stats)
    st = a.stats.cpu().numpy()[-1]
    so = O.stats(a.fitness.cpu().numpy())
    assert st[0] == so[0] and st[2] == so[2] and st[3] == so[3]
