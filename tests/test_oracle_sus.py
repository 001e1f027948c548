"""Oracle pins for selection by stochastic universal sampling after rank scaling
(Algorithm 1 "apply scaling" then "selection"; Section 3.1, Baker's SUS).

The pins are properties that SUS has by construction (each individual is chosen
floor or ceil of its expected number of times; zero-weight individuals never),
the bijectivity of the parent shuffle, and end-to-end behaviour of the GA."""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_1403_4099_amd import synth


def _rank_weights(f):
    # rank 1 = best (fitness desc, index asc); -inf -> 0; all -inf -> 1
    P = len(f)
    order = sorted(range(P), key=lambda p: (-f[p], p))
    w = np.zeros(P, dtype=np.float64)
    for r, p in enumerate(order, start=1):
        w[p] = math.isqrt(2**48 // r) if np.isfinite(f[p]) else 0.0
    return w if w.sum() > 0 else np.ones(P)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 100, 1000, 8190])
def test_shuffle_is_a_bijection(n):
    for seed, gen in ((0, 0), (7, 3), (2**40 + 1, 99)):
        img = [O.shuffle_index(k, n, seed=seed, gen=gen) for k in range(n)]
        assert sorted(img) == list(range(n))
        if n >= 16:
            assert img != list(range(n))


@pytest.mark.parametrize("P,E,seed", [(10, 0, 1), (50, 2, 2), (257, 5, 3), (1000, 10, 4)])
def test_sus_counts_are_floor_or_ceil_of_expectation(P, E, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(P) * 3
    f[rng.integers(0, P, size=P // 10)] = -np.inf
    par = O.sus_parents(f, E=E, seed=seed, gen=5)
    n = 2 * (P - E)
    assert par.shape == (n,) and par.min() >= 0 and par.max() < P
    w = _rank_weights(f)
    expect = n * w / w.sum()
    cnt = np.bincount(par, minlength=P)
    assert np.all(cnt >= np.floor(expect) - 1e-9) and np.all(cnt <= np.ceil(expect) + 1e-9)
    assert np.all(cnt[~np.isfinite(f)] == 0)


def test_all_invalid_population_selects_uniformly():
    P, E = 40, 4
    f = np.full(P, -np.inf)
    par = O.sus_parents(f, E=E, seed=9)
    cnt = np.bincount(par, minlength=P)
    n = 2 * (P - E)
    assert cnt.sum() == n and cnt.min() >= n // P and cnt.max() <= -(-n // P)


def test_offset_and_shuffle_depend_on_generation_and_seed():
    f = np.linspace(5, 1, 64)
    a = O.sus_parents(f, E=2, seed=1, gen=0)
    assert not np.array_equal(a, O.sus_parents(f, E=2, seed=1, gen=1))
    assert not np.array_equal(a, O.sus_parents(f, E=2, seed=2, gen=0))
    assert np.array_equal(a, O.sus_parents(f, E=2, seed=1, gen=0))


def test_breed_with_sus_copies_parent_a_without_crossover_or_mutation():
    rng = np.random.default_rng(5)
    P, N, E = 30, 12, 3
    pop = rng.integers(0, N, size=(P, N), dtype=np.int32)
    f = rng.standard_normal(P)
    out = O.breed(pop, f, E=E, p_cross_thr=0, p_mut_thr=0, seed=3, gen=2, selection=1)
    order = sorted(range(P), key=lambda p: (-f[p], p))
    assert np.array_equal(out[:E], pop[order[:E]])
    par = O.sus_parents(f, E=E, seed=3, gen=2)
    assert np.array_equal(out[E:], pop[par[0::2]])


def test_ga_with_sus_recovers_planted_clusters():
    w = synth.config1()
    C = O.correlate(w.R)
    pop, fit, st, state = O.evolve_term(C, w.P, 400, 0, 1e-5, E=w.elites, seed=w.seed, selection=1)
    lab, fb, _ = O.best(fit, pop)
    f_planted = O.fitness(C, w.planted[None, :])[0]
    assert np.all(np.diff(st[:, 0]) >= 0)
    assert fb >= f_planted - 1e-9
    assert np.array_equal(lab, O.canonical(w.planted))
