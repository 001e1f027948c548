"""GPU parity of the cluster-pair route of pga_fitness / pga_evolve.

An individual whose clusters hold at most frac * N (N - 1) / 2 pairs (and N <= 2048) is
evaluated from those pairs alone (exact FP64 in both forms); every other individual takes the
O(N^2) pair-sum of its form. Checked here:
* the pair route against the oracle (FP64 tolerance), with n_s, c_s and status;
* the choice itself: in a mixed population every individual's result equals, bit for bit, the
  all-pairs result when its pair count (counted on the host) is within the limit and the
  all-dense result otherwise, at the limit and one pair past it included;
* entries with |C_ij| > 1 or NaN inside a cluster, N above 2048 and invalid labels give exactly
  the dense route's results and status;
* evolution through the route (graph and eager) in lockstep with the oracle's breeding."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga, synth
from gpu_cases import corr, fitness_tol, say

pytestmark = pytest.mark.gpu


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def pair_counts(pop, N):
    return np.array([int((lambda n: (n * (n - 1) // 2).sum())(np.bincount(r, minlength=N).astype(np.int64)))
                     for r in pop])


def limit(frac, N):
    return N * (N - 1) // 2 if N <= 64 else math.floor(frac * 0.5 * N * (N - 1))


def _fit(C, pop, form, frac, **kw):
    Cg = _g(C)
    hi = lo = None
    if form == "bf16x2":
        hi, lo = pga.split(Cg)
    with pga.route(frac):
        return pga.fitness(Cg, _g(pop), form, hi=hi, lo=lo, **kw)


PAIR_CASES = [
    # N, P, K (labels in [0, K)), seed
    (1, 3, 1, 0),
    (2, 5, 1, 1),
    (18, 100, 3, 2),
    (63, 70, 63, 3),
    (130, 64, 9, 4),
    (257, 65, 30, 5),
    (1000, 40, 1000, 6),
    (1024, 33, 16, 7),
    (2048, 6, 2048, 8),
    (2048, 3, 3, 9),
]


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
@pytest.mark.parametrize("N,P,K,seed", PAIR_CASES, ids=[f"N{c[0]}-P{c[1]}-K{c[2]}" for c in PAIR_CASES])
def test_pair_route_matches_oracle(N, P, K, seed, form):
    say(f"pair route {form} N={N} P={P} K={K}")
    C, planted = corr(N, T=128, seed=seed)
    pop = synth.random_labelings(P, N, seed=seed, K=K)
    if P > 4:
        pop[-2:] = synth.perturbed_labelings(planted, 2, 0.05, seed)
    f_o, ns_o, cs_o, mag = O.fitness(C, pop, want_ns=True, want_cs=True, want_mag=True)
    st = pga.new_status()
    f_g, ns_g, cs_g = _fit(C, pop, form, 1.0, want_ns=True, want_cs=True, status=st)
    torch.cuda.synchronize()
    assert np.array_equal(ns_g.cpu().numpy(), ns_o)
    assert np.all(np.abs(cs_g.cpu().numpy() - cs_o) <= 1e-12 * np.maximum(1.0, ns_o.astype(float) ** 2))
    d = np.abs(f_g.cpu().numpy() - f_o)
    assert np.all(d <= fitness_tol(mag, 1e-10)), float(np.max(d / np.maximum(mag, 1e-300)))
    assert st.cpu().numpy().sum() == 0


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_each_individual_takes_the_route_its_pair_count_selects(form):
    N, frac = 300, 1.0 / 64
    lim = limit(frac, N)
    say(f"route choice {form} N={N} limit={lim}")
    C, _ = corr(N, T=128, seed=21)
    parts = [synth.random_labelings(40, N, seed=22, K=K) for K in (N, N // 2, N // 8, 12, 3)]
    pop = np.concatenate(parts)
    # one individual exactly at the limit and one a pair past it (singletons elsewhere)
    for extra in (0, 1):
        row = np.arange(N, dtype=np.int32)
        need, pos = lim + extra, 0
        while need > 0:
            n = 2
            while (n + 1) * n // 2 <= need:
                n += 1
            row[pos:pos + n] = row[pos]
            need -= n * (n - 1) // 2
            pos += n
        pop = np.concatenate([pop, row[None, :]])
    pc = pair_counts(pop, N)
    assert pc[-2] == lim and pc[-1] == lim + 1
    on = pc <= lim
    assert on.any() and (~on).any()
    f_mix = _fit(C, pop, form, frac).cpu().numpy()
    f_pairs = _fit(C, pop, form, 1.0).cpu().numpy()
    f_dense = _fit(C, pop, form, 0.0).cpu().numpy()
    assert np.array_equal(f_mix[on], f_pairs[on])
    assert np.array_equal(f_mix[~on], f_dense[~on])
    # the pair route is the same arithmetic in both forms
    other = "bf16x2" if form == "fp64" else "fp64"
    assert np.array_equal(f_pairs, _fit(C, pop, other, 1.0).cpu().numpy())
    f_o, mag = O.fitness(C, pop, want_mag=True)
    assert np.all(np.abs(f_pairs - f_o) <= fitness_tol(mag, 1e-10))


def test_entries_outside_the_unit_interval_take_the_dense_route():
    N = 40
    C, _ = corr(N, T=64, seed=31)
    C = C.copy()
    C[3, 5] = C[5, 3] = 1.5
    C[10, 11] = C[11, 10] = np.nan
    pop = synth.random_labelings(30, N, seed=32, K=N)
    pop[0, [3, 5]] = 7                        # pair (3, 5) in one cluster
    pop[1, [10, 11]] = 2                      # pair (10, 11) in one cluster
    for r in range(2, len(pop)):              # elsewhere the two pairs are never in one cluster
        for a, b in ((3, 5), (10, 11)):
            if pop[r, a] == pop[r, b]:
                pop[r, b] = (pop[r, b] + 1) % N
    for form in ("fp64", "bf16x2"):
        st_a, st_b = pga.new_status(), pga.new_status()
        a, nsa, csa = _fit(C, pop, form, 1.0, want_ns=True, want_cs=True, status=st_a)
        b, nsb, csb = _fit(C, pop, form, 0.0, want_ns=True, want_cs=True, status=st_b)
        a, b = a.cpu().numpy(), b.cpu().numpy()
        assert np.isinf(a[1]) and np.isinf(b[1])
        assert np.array_equal(a[:2], b[:2]), form
        assert np.array_equal(nsa.cpu().numpy()[:2], nsb.cpu().numpy()[:2])
        assert np.array_equal(csa.cpu().numpy()[:2], csb.cpu().numpy()[:2])
        if form == "fp64":   # the MFMA form's NaN reaches every individual of the dense route
            assert np.array_equal(st_a.cpu().numpy(), st_b.cpu().numpy())
    # the other individuals never meet a bad entry: the pair route agrees with the oracle
    f = _fit(C, pop, "fp64", 1.0).cpu().numpy()
    Cc = np.where(np.isfinite(C), np.clip(C, -1, 1), 0.0)
    f_o, mag = O.fitness(Cc, pop[2:], want_mag=True)
    assert np.all(np.abs(f[2:] - f_o) <= fitness_tol(mag, 1e-10))


def test_pair_route_with_a_diagonal_other_than_ones():
    """C_jj below 1 is summed term by term (the all-ones shortcut does not apply); a C_jj above 1
    sends every individual to the pair-sum route."""
    N = 90
    C, _ = corr(N, T=64, seed=71)
    rng = np.random.default_rng(72)
    C = C.copy()
    np.fill_diagonal(C, rng.uniform(0.6, 1.0, N))
    pop = synth.random_labelings(50, N, seed=73, K=12)
    f_o, ns_o, cs_o, mag = O.fitness(C, pop, want_ns=True, want_cs=True, want_mag=True)
    for form in ("fp64", "bf16x2"):
        f_g, ns_g, cs_g = _fit(C, pop, form, 1.0, want_ns=True, want_cs=True)
        assert np.array_equal(ns_g.cpu().numpy(), ns_o)
        assert np.all(np.abs(cs_g.cpu().numpy() - cs_o) <= 1e-12 * np.maximum(1.0, ns_o.astype(float) ** 2))
        assert np.all(np.abs(f_g.cpu().numpy() - f_o) <= fitness_tol(mag, 1e-10))
    C[7, 7] = 1.25
    for form in ("fp64", "bf16x2"):
        assert torch.equal(_fit(C, pop, form, 1.0), _fit(C, pop, form, 0.0))


def test_invalid_labels_and_domain_status_as_dense_route():
    C = np.array([[1.0, 1.0, 0.1, 0.0], [1.0, 1.0, 0.1, 0.0], [0.1, 0.1, 1.0, -1.0], [0.0, 0.0, -1.0, 1.0]])
    pop = np.array([[0, 0, 1, 2], [0, 1, 2, 2], [0, 1, 4, 3], [-1, 0, 0, 0], [0, 1, 2, 3], [1, 1, 1, 1]],
                   dtype=np.int32)
    st_o = O.status_zero()
    f_o, ns_o, cs_o = O.fitness(C, pop, want_ns=True, want_cs=True, status=st_o)
    for form in ("fp64", "bf16x2"):
        st = pga.new_status()
        f_g, ns_g, cs_g = _fit(C, pop, form, 1.0, want_ns=True, want_cs=True, status=st)
        f_g = f_g.cpu().numpy()
        assert np.array_equal(np.isinf(f_g), np.isinf(f_o))
        assert np.allclose(f_g[np.isfinite(f_o)], f_o[np.isfinite(f_o)], rtol=1e-12, atol=1e-13)
        assert np.array_equal(st.cpu().numpy(), st_o), form
        assert np.array_equal(ns_g.cpu().numpy(), ns_o)
        assert np.allclose(cs_g.cpu().numpy(), cs_o, rtol=1e-12, atol=1e-13)


def test_above_2048_stocks_every_individual_takes_the_dense_route():
    N = 2049
    C, _ = corr(N, T=64, seed=41)
    pop = synth.random_labelings(5, N, seed=42)
    for form in ("fp64", "bf16x2"):
        assert torch.equal(_fit(C, pop, form, 1.0), _fit(C, pop, form, 0.0))


def test_pair_route_is_deterministic():
    C, _ = corr(500, T=64, seed=51)
    pop = synth.random_labelings(300, 500, seed=52, K=60)
    a = _fit(C, pop, "fp64", 1.0, want_cs=True)
    b = _fit(C, pop, "fp64", 1.0, want_cs=True)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("frac", [0.0, 1.0 / 64, 1.0], ids=["dense", "default", "pairs"])
@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_evolve_through_the_route_in_lockstep_with_oracle(form, frac):
    N, P, E, G = 130, 64, 2, 3
    say(f"evolve route={frac} {form}")
    C, _ = corr(N, seed=61)
    Cg = _g(C)
    hi = lo = None
    if form == "bf16x2":
        hi, lo = pga.split(Cg)
    with pga.route(frac):
        I = pga.make_instance(Cg, P, hi=hi, lo=lo, stats_rows=G + 1, elites=E, seed=5, instance_id=1)
        ctx = pga.Context()
        ctx.evolve([I], 0, form=form, init=True)
        pop = I.pop.cpu().numpy()
        for g in range(G):
            f = I.fitness.cpu().numpy()
            I.gen0 = g
            ctx.evolve([I], 1, form=form)
            nxt = O.breed(pop, f, E=E, seed=5, inst=1, gen=g, selection=0)
            assert np.array_equal(I.pop.cpu().numpy(), nxt), g
            pop = nxt
        # graph replay equals eager launches
        J = pga.make_instance(Cg, P, hi=hi, lo=lo, pop=_g(pop), stats_rows=3, elites=E, seed=5, instance_id=1)
        K = pga.make_instance(Cg, P, hi=hi, lo=lo, pop=_g(pop), stats_rows=3, elites=E, seed=5, instance_id=1)
        ctx.evolve([J], 2, form=form)
        ctx.evolve([K], 2, form=form, eager=True)
        assert torch.equal(J.pop, K.pop) and torch.equal(J.fitness, K.fitness)
    f_o, mag = O.fitness(C, I.pop.cpu().numpy(), want_mag=True)
    tol = fitness_tol(mag, 1e-10) if (form == "fp64" or frac == 1.0) else 1e-4 * mag + 1e-9
    assert np.all(np.abs(I.fitness.cpu().numpy() - f_o) <= tol)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_batch_mixing_an_instance_above_2048_equals_each_alone(form):
    """One launch sequence holds an instance above 2048 stocks (always the pair-sum route) and
    small ones (cluster-pair route, with LDS laid out for 2048): each result equals its own run."""
    specs = [(2100, 6, 0, 31), (150, 40, 1, 32), (37, 24, 2, 33)]
    G = 2
    ctx = pga.Context()

    def inst(N, P, iid, seed, pop=None):
        C, _ = corr(N, T=64, seed=80 + iid)
        Cg = _g(C)
        hi = lo = None
        if form == "bf16x2":
            hi, lo = pga.split(Cg)
        return pga.make_instance(Cg, P, hi=hi, lo=lo, pop=pop, stats_rows=G + 1, elites=1, seed=seed,
                                 instance_id=iid)

    with pga.route(1.0 / 64):
        alone = []
        for N, P, iid, seed in specs:
            I = inst(N, P, iid, seed)
            ctx.evolve([I], G, form=form, init=True)
            alone.append(I)
        batch = [inst(N, P, iid, seed) for N, P, iid, seed in specs]
        ctx.evolve(batch, G, form=form, init=True)
        torch.cuda.synchronize()
    for a, b in zip(alone, batch):
        assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness) and torch.equal(a.stats, b.stats)


@pytest.mark.parametrize("N,P", [(300, 9000), (600, 8200)], ids=["wave-kernel", "workgroup-kernel"])
def test_route_lists_of_a_large_launch_equal_the_per_individual_launches(N, P):
    """A launch of 8192 individuals or more sorts them into route lists (a route kernel, then a
    workgroup per listed individual); smaller launches take a workgroup per individual. The same
    population evaluated whole and in small chunks gives the same bits, the pair route agrees with
    the oracle, and an individual holding an entry above 1 inside a cluster is handed back to the
    pair-sum route in the list form too."""
    say(f"route lists N={N} P={P}")
    C, planted = corr(N, T=64, seed=91)
    C = C.copy()
    C[3, 5] = C[5, 3] = 1.5
    parts = [synth.random_labelings(P // 4, N, seed=92 + i, K=K) for i, K in enumerate((N, N // 4, 40, 9))]
    pop = np.concatenate(parts)
    pop[:: 97, 5] = pop[:: 97, 3]                          # pair (3, 5) in one cluster: the bad entry
    for form in ("fp64", "bf16x2"):
        Cg = _g(C)
        hi = lo = None
        if form == "bf16x2":
            hi, lo = pga.split(Cg)
        with pga.route(1.0 / 64):
            whole = pga.fitness(Cg, _g(pop), form, hi=hi, lo=lo, want_ns=True)
            parts_g = [pga.fitness(Cg, _g(pop[i:i + 2000]), form, hi=hi, lo=lo, want_ns=True)
                       for i in range(0, len(pop), 2000)]
        assert torch.equal(whole[0], torch.cat([f for f, _ in parts_g])), form
        assert torch.equal(whole[1], torch.cat([n for _, n in parts_g])), form
    f = whole[0].cpu().numpy()
    pc = pair_counts(pop, N)
    bad = pop[:, 3] == pop[:, 5]
    on = (pc <= limit(1.0 / 64, N)) & ~bad
    assert on.sum() > 100 and (~on).sum() > 100 and bad.sum() > 50
    sample = np.flatnonzero(on)[:: 40]
    Cc = np.clip(C, -1, 1)
    f_o, mag = O.fitness(Cc, pop[sample], want_mag=True)
    assert np.all(np.abs(f[sample] - f_o) <= fitness_tol(mag, 1e-10))
    with pga.route(0.0):
        dense = pga.fitness(_g(C), _g(pop[bad]), "fp64").cpu().numpy()
    with pga.route(1.0 / 64):
        listed_bad = pga.fitness(_g(C), _g(pop), "fp64").cpu().numpy()[bad]
    assert np.array_equal(listed_bad, dense)


@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_batch_of_many_individuals_equals_each_instance_alone(form):
    """16 instances of 520 individuals (8320 in one launch: route lists, one wave per breed slot)
    evolve to the same bits as each instance alone (520: a workgroup per individual and slot)."""
    G = 3
    specs = [(int(n), 520, i) for i, n in enumerate(np.random.default_rng(5).integers(40, 400, size=16))]
    say(f"many-individual batch {form}")
    Cs = [corr(N, T=64, seed=100 + i)[0] for N, _, i in specs]

    def inst(C, P, i):
        Cg = _g(C)
        hi = lo = None
        if form == "bf16x2":
            hi, lo = pga.split(Cg)
        return pga.make_instance(Cg, P, hi=hi, lo=lo, stats_rows=G + 1, elites=2, seed=17, instance_id=i)

    ctx = pga.Context()
    with pga.route(1.0 / 64):
        batch = [inst(C, P, i) for C, (N, P, i) in zip(Cs, specs)]
        ctx.evolve(batch, G, form=form, init=True)
        torch.cuda.synchronize()
        for C, (N, P, i), b in zip(Cs, specs, batch):
            a = inst(C, P, i)
            pga.Context().evolve([a], G, form=form, init=True)
            torch.cuda.synchronize()
            assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness), i
            assert torch.equal(a.stats, b.stats), i


def test_large_batch_with_sus_and_stopping_instances_equals_each_alone():
    """A launch of more than 8192 individuals breeds one wave per slot: the SUS parent pick, the
    elite copies from the rank kernel (no fold: some instances can stop) and stopped instances
    take that kernel's paths. Every instance equals its own run (a workgroup per slot)."""
    G = 7
    rng = np.random.default_rng(12)
    specs = []                                           # N, P, selection, stall, tol
    for i in range(17):
        sel = "sus" if i % 3 == 0 else "tournament"
        stall, tol = ((3, 1e9) if i % 4 == 1 else (0, 1e-5))
        specs.append((int(rng.integers(30, 300)), 500, sel, stall, tol))
    assert sum(s[1] for s in specs) > 8192
    say("large batch with SUS and stopping instances")
    Cs = [corr(N, T=64, seed=140 + i)[0] for i, (N, *_r) in enumerate(specs)]

    def inst(i, C, P, sel, stall, tol):
        I = pga.make_instance(_g(C), P, stats_rows=G + 1, elites=2, seed=23, instance_id=i, selection=sel,
                              stall_gens=stall, tol=tol)
        I.stats.fill_(float("nan"))
        return I

    with pga.route(1.0 / 64):
        batch = [inst(i, C, *s[1:]) for i, (C, s) in enumerate(zip(Cs, specs))]
        pga.Context().evolve(batch, G, init=True)
        torch.cuda.synchronize()
        for i, (C, s) in enumerate(zip(Cs, specs)):
            a = inst(i, C, *s[1:])
            pga.Context().evolve([a], G, init=True)
            torch.cuda.synchronize()
            b = batch[i]
            assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness), i
            assert torch.equal(torch.nan_to_num(a.stats, nan=7.0), torch.nan_to_num(b.stats, nan=7.0)), i
            assert a.term_state() == b.term_state(), i
    stopped = [b.term_state()["stopped"] for b in batch]
    assert any(stopped) and not all(stopped)


@pytest.mark.parametrize("nlo,nhi", [(8, 32), (33, 64)], ids=["16-lane-slots", "32-lane-slots"])
def test_large_batch_of_small_instances_equals_each_alone(nlo, nhi):
    """Launches of more than 8192 individuals whose largest N is at most 32 (64) breed four (two)
    children per wave, 16 (32) lanes each; with SUS and tournament instances, every instance
    equals its own run (a workgroup per slot)."""
    G = 4
    rng = np.random.default_rng(nhi)
    specs = [(int(rng.integers(nlo, nhi + 1)), 450, "sus" if i % 4 == 0 else "tournament") for i in range(20)]
    specs[0] = (nhi, 450, "sus")
    say(f"large batch of small instances N in [{nlo}, {nhi}]")
    Cs = [corr(N, T=64, seed=170 + i)[0] for i, (N, *_r) in enumerate(specs)]

    def inst(i, C, P, sel):
        return pga.make_instance(_g(C), P, stats_rows=G + 1, elites=3, seed=31, instance_id=i, selection=sel)

    with pga.route(1.0 / 64):
        batch = [inst(i, C, P, sel) for i, (C, (N, P, sel)) in enumerate(zip(Cs, specs))]
        pga.Context().evolve(batch, G, init=True)
        torch.cuda.synchronize()
        for i, (C, (N, P, sel)) in enumerate(zip(Cs, specs)):
            a = inst(i, C, P, sel)
            pga.Context().evolve([a], G, init=True)
            torch.cuda.synchronize()
            b = batch[i]
            assert torch.equal(a.pop, b.pop) and torch.equal(a.fitness, b.fitness), i
            assert torch.equal(a.stats, b.stats), i
