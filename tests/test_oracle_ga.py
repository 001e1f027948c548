"""Pins for the oracle's genetic operators and loop (Section 3.1, Algorithm 1)."""
import numpy as np
import pytest

import oracle as O
from paper_1403_4099_amd import synth

TAG_SEL, TAG_XOV, TAG_MUT = 1, 2, 3


def _draw(w0, c, gen, tag, seed=0, inst=0):
    return O.philox([w0, c, gen, tag | (inst << 4)], [seed & 0xFFFFFFFF, seed >> 32])


def _scale(w, m):
    return (int(w) * m) >> 32


def _distinct_pop(P, N):
    # row p is identifiable from any of its genes: gene j = (p + j * P) mod N with N > P
    assert N > P
    return ((np.arange(P)[:, None] + np.arange(N)[None, :] * P) % N).astype(np.int32)


def test_tournament_with_index_fitness_picks_larger_index():
    P, N, E = 40, 101, 0
    pop = _distinct_pop(P, N)
    f = np.arange(P, dtype=np.float64)          # fitness = index, all distinct
    out = O.breed(pop, f, E=E, p_cross_thr=0, p_mut_thr=0, seed=99, gen=5)
    for c in range(P):
        w = _draw(0, c, 5, TAG_SEL, seed=99)
        a = max(_scale(w[0], P), _scale(w[1], P))
        assert np.array_equal(out[c], pop[a])


def test_tournament_ties_go_to_lower_index_and_inf_loses():
    P, N = 30, 61
    pop = _distinct_pop(P, N)
    f = np.zeros(P)
    f[::3] = -np.inf
    out = O.breed(pop, f, E=0, p_cross_thr=0, p_mut_thr=0, seed=3, gen=1)
    for c in range(P):
        w = _draw(0, c, 1, TAG_SEL, seed=3)
        a, b = _scale(w[0], P), _scale(w[1], P)
        fa, fb = f[a], f[b]
        win = a if fa > fb else b if fb > fa else min(a, b)
        assert np.array_equal(out[c], pop[win])


def test_elites_are_the_fittest_copied_unchanged():
    P, N, E = 50, 77, 5
    rng = np.random.default_rng(0)
    pop = rng.integers(0, N, size=(P, N)).astype(np.int32)
    f = rng.standard_normal(P)
    f[[3, 9]] = f.max() + 1.0                  # a tie at the top: lower index first
    f[11] = -np.inf
    out = O.breed(pop, f, E=E, seed=1, gen=0)
    order = sorted(range(P), key=lambda p: (-f[p], p))
    for e in range(E):
        assert np.array_equal(out[e], pop[order[e]])
    assert order[0] == 3 and order[1] == 9


def test_uniform_crossover_takes_genes_from_both_parents():
    P, N = 20, 1000
    pop = np.zeros((P, N), dtype=np.int32)
    pop[:, :] = np.arange(P)[:, None]          # parent identified by its constant label
    f = np.arange(P, dtype=np.float64)
    out = O.breed(pop, f, E=0, p_cross_thr=2**32 - 1, p_mut_thr=0, seed=11, gen=2)
    fracs = []
    for c in range(P):
        w = _draw(0, c, 2, TAG_SEL, seed=11)
        A = max(_scale(w[0], P), _scale(w[1], P))
        B = max(_scale(w[2], P), _scale(w[3], P))
        assert set(np.unique(out[c])) <= {A, B}
        if A != B:
            fromB = out[c] == B
            fracs.append(fromB.mean())
            # the bit rule, checked gene by gene on the first 300 genes
            for j in range(300):
                wb = _draw(1 + j // 128, c, 2, TAG_XOV, seed=11)
                r = j % 128
                bit = (int(wb[r // 32]) >> (r % 32)) & 1
                assert fromB[j] == bool(bit)
    assert len(fracs) > 5
    assert abs(np.mean(fracs) - 0.5) < 0.05


def test_crossover_probability():
    P, N = 3000, 4
    pop = np.zeros((P, N), dtype=np.int32)
    f = np.zeros(P)
    thr = int(0.9 * 2**32)
    fired = sum(int(_draw(0, c, 0, TAG_XOV)[0]) < thr for c in range(P))
    assert abs(fired / P - 0.9) < 4 * np.sqrt(0.09 / P)


def test_mutation_rate_is_one_over_n():
    P, N, E = 400, 150, 2
    pop = np.tile(np.arange(N, dtype=np.int32) % 7, (P, 1))
    f = np.zeros(P)
    out = O.breed(pop, f, E=E, p_cross_thr=0, seed=21, gen=3)
    n = (P - E) * N
    changed = int(np.sum(out[E:] != pop[E:]))
    # mutation fires w.p. ~1/N; the new label is uniform on [0, N), so it equals the old one w.p. 1/N
    p_fire = O.mut_thr(N) / 2**32
    p_change = p_fire * (1 - 1 / N)
    sd = np.sqrt(n * p_change * (1 - p_change))
    assert abs(changed - n * p_change) < 5 * sd
    assert out.min() >= 0 and out.max() < N


def test_evolve_best_is_monotone_and_resume_is_exact():
    w = synth.config1()
    C = O.correlate(w.R)
    pop_a, fit_a, st_a = O.evolve(C, P=60, G=30, E=2, seed=5)
    assert np.all(np.diff(st_a[:, 0]) >= 0.0)
    pop_b, fit_b, st_b = O.evolve(C, P=60, G=12, E=2, seed=5)
    pop_c, fit_c, st_c = O.evolve(C, P=60, G=18, E=2, seed=5, gen0=12, pop=pop_b)
    assert np.array_equal(pop_a, pop_c)
    assert np.array_equal(fit_a, fit_c)
    assert np.array_equal(st_a[12:], st_c)
    assert np.array_equal(st_a[:12], st_b[:12])


def test_evolve_without_elites_is_allowed_and_stats_are_consistent():
    w = synth.config1()
    C = O.correlate(w.R)
    pop, fit, st = O.evolve(C, P=20, G=5, E=0, seed=2)
    s = O.stats(fit)
    assert np.array_equal(s, st[-1])
    assert st[-1, 0] == fit.max() and st[-1, 3] == int(np.argmax(fit))


def test_recovers_planted_clusters_config1():
    """The 18-stock configuration: the GA's best labeling is the planted 8/6/4 partition."""
    w = synth.config1()
    C = O.correlate(w.R)
    pop, fit, st = O.evolve(C, P=w.P, G=w.G, E=w.elites, seed=w.seed)
    lab, bf, idx = O.best(fit, pop)
    assert np.array_equal(lab, O.canonical(w.planted))
    assert bf == pytest.approx(O.fitness(C, w.planted[None, :])[0], rel=1e-14)


def test_ga_matches_brute_force_on_small_sampled_matrix():
    rng = np.random.default_rng(17)
    R, planted = synth.one_factor_returns([4, 3], [0.6, 0.5], 2, 400, rng)
    C = O.correlate(R)
    bf, blab, nbest, _ = O.brute_force(C)
    assert nbest == 1
    pop, fit, st = O.evolve(C, P=60, G=60, E=2, seed=0)
    lab, f, _ = O.best(fit, pop)
    assert np.array_equal(lab, O.canonical(blab))
    assert f == pytest.approx(bf, rel=1e-14)


def test_best_and_canonical():
    f = np.array([0.5, 2.0, 2.0, -np.inf])
    pop = np.array([[0, 0, 0], [2, 2, 1], [0, 1, 2], [0, 0, 0]], dtype=np.int32)
    lab, bf, idx = O.best(f, pop)
    assert idx == 1 and bf == 2.0 and list(lab) == [0, 0, 1]
    assert list(O.canonical(np.array([4, 3, 4, 0, 3], dtype=np.int32))) == [0, 1, 0, 2, 1]


def _clusters(lab):
    groups = {}
    for i, l in enumerate(lab):
        groups.setdefault(int(l), []).append(i)
    return {tuple(v) for v in groups.values()}


def test_recovers_planted_clusters_config2():
    """N=100 with 10 noise stocks, 500 generations: every planted cluster with loading
    g >= 0.35 is found exactly; no cluster is merged with another (the label held by
    most of a planted cluster's stocks is held by no stock outside it) and that label
    holds at least 60% of the cluster; the best labeling reaches 98% of the planted
    likelihood. (The two weakest clusters of this draw, g = 0.22 and 0.28, are still
    being assembled at generation 500 with tournament-2 / uniform crossover: 7 of 10
    and 4 of 6 stocks.)"""
    w = synth.config2()
    C = O.correlate(w.R)
    pop, fit, st = O.evolve(C, P=w.P, G=w.G, E=w.elites, seed=w.seed)
    lab, bf, _ = O.best(fit, pop)
    found = _clusters(lab)
    for k, gk in enumerate(w.g):
        members = np.nonzero(w.planted == k)[0]
        if gk >= 0.35:
            assert tuple(int(i) for i in members) in found
        vals, cnts = np.unique(lab[members], return_counts=True)
        top = vals[np.argmax(cnts)]
        assert cnts.max() >= 0.6 * len(members)
        assert np.all(np.isin(np.nonzero(lab == top)[0], members))
    assert bf >= 0.98 * O.fitness(C, w.planted[None, :])[0]
    assert np.all(np.diff(st[:, 0]) >= 0.0)
