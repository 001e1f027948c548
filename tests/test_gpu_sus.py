"""GPU parity of selection by stochastic universal sampling (PGA_SELECT_SUS) against
the CPU oracle: lockstep generations (the oracle breeds from the GPU's population and
fitness; the GPU's next population must match bit for bit), and batching."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga
from gpu_cases import corr, say

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _inst(C, P, G, form="fp64", pop=None, **kw):
    Cg = _g(C)
    hi = lo = None
    if form == "bf16x2":
        hi, lo = pga.split(Cg)
    return pga.make_instance(Cg, P, hi=hi, lo=lo, pop=None if pop is None else _g(pop), stats_rows=G + 1,
                             selection="sus", **kw)


CASES = [
    # N, P, E, generations, form, invalid rows in the start population
    (18, 100, 2, 8, "fp64", 0),
    (130, 257, 5, 3, "fp64", 0),
    (40, 1500, 10, 2, "fp64", 0),
    (60, 300, 3, 3, "fp64", 40),
    (37, 90, 0, 3, "bf16x2", 0),
]


@pytest.mark.parametrize("N,P,E,G,form,bad", CASES, ids=[f"N{c[0]}-P{c[1]}-E{c[2]}-{c[4]}-bad{c[5]}" for c in CASES])
def test_sus_breed_lockstep_with_oracle(N, P, E, G, form, bad):
    say(f"SUS lockstep N={N} P={P} E={E} {form} bad={bad}")
    C, _ = corr(N, seed=5)
    pop0 = O.init_pop(N, P, seed=21, inst=4)
    if bad:
        pop0[np.random.default_rng(1).choice(P, size=bad, replace=False), 0] = N   # out of range: fitness -inf
    ctx = pga.Context()
    I = _inst(C, P, 1, form=form, pop=pop0, elites=E, seed=21, instance_id=4)
    for g in range(G):
        pop_g = I.pop.clone()
        f_g = pga.fitness(I.C, pop_g, form, hi=I.hi, lo=I.lo)
        I.gen0 = g
        ctx.evolve([I], 1, form=form, eager=(g % 2 == 1))
        nxt = O.breed(pop_g.cpu().numpy(), f_g.cpu().numpy(), E=E, seed=21, inst=4, gen=g, selection=1)
        assert np.array_equal(I.pop.cpu().numpy(), nxt), f"generation {g}"
        if bad and g == 0:
            assert (~torch.isfinite(f_g)).sum().item() == bad


def test_sus_batched_with_tournament_instances_equals_each_alone():
    say("SUS in a batch with tournament instances")
    specs = [(18, 100, "sus"), (70, 64, "tournament"), (130, 300, "sus"), (33, 16, "tournament")]
    G = 6
    Cs = [corr(N, seed=20 + i)[0] for i, (N, _, _) in enumerate(specs)]

    def make(i, C, P, sel):
        return pga.make_instance(_g(C), P, stats_rows=G + 1, seed=8, instance_id=i, selection=sel)

    alone = []
    for i, (C, (N, P, sel)) in enumerate(zip(Cs, specs)):
        I = make(i, C, P, sel)
        pga.Context().evolve([I], G, init=True)
        alone.append(I)
    batch = [make(i, C, P, sel) for i, (C, (N, P, sel)) in enumerate(zip(Cs, specs))]
    ctx = pga.Context()
    ctx.evolve(batch, G, init=True)
    torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a.pop, b.pop) and torch.equal(a.stats[: G + 1], b.stats[: G + 1])
    # and the SUS instances followed the oracle's free-running SUS GA where fitness ties do not intervene
    C0 = Cs[0]
    pop_o, fit_o, st_o, _ = O.evolve_term(C0, 100, G, 0, 0.0, seed=8, inst=0, selection=1)
    assert np.array_equal(batch[0].pop.cpu().numpy(), pop_o)
