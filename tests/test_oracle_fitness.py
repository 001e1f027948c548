"""Pins for the oracle's likelihood (Eqs. 5, 6, 8) against facts the paper and mathematics fix.

None of these re-types Eq. 8: the closed form uses numpy's log-determinant,
n_s uses numpy bincount, c_s uses a numpy one-hot matrix product, and the rest
are invariants, special cases and brute force.
"""
import numpy as np
import pytest

import oracle as O
from paper_1403_4099_amd import synth


def _canon(lab):
    return O.canonical(np.asarray(lab, dtype=np.int32))


@pytest.mark.parametrize("sizes,rhos,n_single", [
    ([2], [0.5], 0),
    ([3, 2], [0.2, 0.8], 1),
    ([8, 6, 4], [0.3, 0.5, 0.7], 0),
    ([5, 5, 3, 2], [0.05, 0.9, -0.2, 0.6], 4),
    ([40], [0.45], 10),
])
def test_block_matrix_closed_form(sizes, rhos, n_single):
    """Exact compound-symmetric blocks with the planted labeling: L_c = -1/2 log det C."""
    C, planted = synth.block_correlation(sizes, rhos, n_single)
    sign, logdet = np.linalg.slogdet(C)
    assert sign > 0
    L = O.fitness(C, planted[None, :])[0]
    assert L == pytest.approx(-0.5 * logdet, rel=1e-12, abs=1e-13)
    # same with the stocks shuffled
    rng = np.random.default_rng(7)
    perm = rng.permutation(C.shape[0])
    L2 = O.fitness(C[np.ix_(perm, perm)], planted[perm][None, :])[0]
    assert L2 == pytest.approx(L, rel=1e-13, abs=1e-14)


@pytest.mark.parametrize("rho", [-0.95, -0.5, -0.01, 0.0, 0.01, 0.3, 0.9, 0.999])
def test_two_stocks_closed_form(rho):
    C = np.array([[1.0, rho], [rho, 1.0]])
    L_pair = O.fitness(C, np.array([[0, 0]]))[0]
    L_pair_relabelled = O.fitness(C, np.array([[1, 1]]))[0]
    L_single = O.fitness(C, np.array([[0, 1]]))[0]
    expect = -0.5 * np.log1p(-rho * rho)
    assert L_pair == pytest.approx(expect, rel=1e-12, abs=1e-15)
    assert L_pair_relabelled == L_pair
    assert L_single == 0.0


def test_identity_gives_zero_exactly():
    """Uncorrelated stocks: c_s = n_s for every cluster, so every term vanishes (text after Eq. 8)."""
    for N in (1, 2, 7, 33):
        C = np.eye(N)
        pop = synth.random_labelings(20, N, seed=N, K=max(1, N // 3))
        fit = O.fitness(C, pop)
        assert np.all(fit == 0.0)


def test_all_singletons_zero():
    C = synth.random_symmetric_unit_diag(25, seed=3)
    lab = np.arange(25, dtype=np.int32)[None, :]
    assert O.fitness(C, lab)[0] == 0.0


def _sample_corr(N, T, seed):
    rng = np.random.default_rng(seed)
    sizes = [N // 3, N // 4]
    g = [0.4, 0.6]
    R, planted = synth.one_factor_returns(sizes, g, N - sum(sizes), T, rng)
    return np.corrcoef(R), planted


def test_ns_matches_bincount_and_cs_matches_onehot_product():
    C, _ = _sample_corr(30, 200, seed=1)
    pop = synth.random_labelings(50, 30, seed=2, K=8)
    fit, ns, cs = O.fitness(C, pop, want_ns=True, want_cs=True)
    for p in range(pop.shape[0]):
        assert np.array_equal(ns[p], np.bincount(pop[p], minlength=30))
        Y = np.zeros((30, 30))
        Y[np.arange(30), pop[p]] = 1.0
        cs_ref = np.einsum("is,ij,js->s", Y, C, Y)
        np.testing.assert_allclose(cs[p], cs_ref, rtol=1e-13, atol=1e-13)


def test_label_value_permutation_invariance():
    C, _ = _sample_corr(40, 300, seed=4)
    pop = synth.random_labelings(30, 40, seed=5, K=10)
    fit, mag = O.fitness(C, pop, want_mag=True)
    rng = np.random.default_rng(6)
    relabel = rng.permutation(40).astype(np.int32)
    fit2 = O.fitness(C, relabel[pop])
    assert np.all(np.abs(fit2 - fit) <= 1e-13 * mag + 1e-15)


def test_stock_permutation_invariance():
    C, _ = _sample_corr(40, 300, seed=8)
    pop = synth.random_labelings(30, 40, seed=9, K=6)
    fit, mag = O.fitness(C, pop, want_mag=True)
    perm = np.random.default_rng(10).permutation(40)
    fit2 = O.fitness(C[np.ix_(perm, perm)], pop[:, perm])
    assert np.all(np.abs(fit2 - fit) <= 1e-12 * mag + 1e-15)


def test_likelihood_is_nonnegative_on_valid_labelings():
    """Each cluster term is convex in c_s with minimum 0 at c_s = n_s, so L_c >= 0."""
    C, _ = _sample_corr(60, 100, seed=11)
    pop = synth.random_labelings(200, 60, seed=12, K=5)
    fit = O.fitness(C, pop)
    assert np.all(np.isfinite(fit))
    assert np.all(fit >= -1e-12)


def test_literal_form_for_anticorrelated_cluster():
    """c_s < n_s keeps the literal Eq. 8 (positive term), not a clamp to zero."""
    rho = -0.4
    C = np.array([[1.0, rho, 0.0], [rho, 1.0, 0.0], [0.0, 0.0, 1.0]])
    L = O.fitness(C, np.array([[0, 0, 2]]))[0]
    assert L > 0.0
    assert L == pytest.approx(-0.5 * np.log1p(-rho * rho), rel=1e-12)


def test_domain_and_label_errors():
    # two identical stocks: c_s = n_s^2 for the pair -> outside the domain
    C = np.array([[1.0, 1.0, 0.1], [1.0, 1.0, 0.1], [0.1, 0.1, 1.0]])
    st = O.status_zero()
    fit = O.fitness(C, np.array([[0, 0, 1], [0, 1, 2], [0, 0, 0]]), status=st)
    assert fit[0] == -np.inf
    assert np.isfinite(fit[1]) and fit[1] == 0.0
    assert np.isfinite(fit[2])
    assert list(st[:4]) == [0, 1, 0, 1]
    # perfectly anti-correlated pair: c_s = 0 -> outside the domain
    C2 = np.array([[1.0, -1.0], [-1.0, 1.0]])
    st = O.status_zero()
    assert O.fitness(C2, np.array([[1, 1]]), status=st)[0] == -np.inf
    assert list(st[:4]) == [0, 1, 0, 1]
    # labels outside [0, N)
    st = O.status_zero()
    fit = O.fitness(np.eye(4), np.array([[0, 1, 4, 0], [-1, 0, 0, 0], [3, 3, 3, 3]]), status=st)
    assert fit[0] == -np.inf and fit[1] == -np.inf and fit[2] == 0.0
    assert list(st[:4]) == [2, 0, 0, 2]


def _bell():
    rows = np.loadtxt(__file__.replace("test_oracle_fitness.py", "golden/bell_numbers.txt"), dtype=np.int64)
    return dict(rows)


def test_brute_force_visits_every_partition():
    bell = _bell()
    for N in range(1, 11):
        C = np.eye(N)
        _, _, _, cnt = O.brute_force(C)
        assert cnt == bell[N]


@pytest.mark.parametrize("sizes,rhos,n_single,seed", [
    ([4, 3, 2], [0.5, 0.6, 0.7], 0, 0),
    ([3, 3], [0.4, 0.8], 1, 1),
    ([5, 2], [0.3, 0.9], 1, 2),
])
def test_brute_force_argmax_is_planted_on_exact_blocks(sizes, rhos, n_single, seed):
    C, planted = synth.block_correlation(sizes, rhos, n_single)
    perm = np.random.default_rng(seed).permutation(C.shape[0])
    C = C[np.ix_(perm, perm)]
    planted = planted[perm]
    bf, lab, nbest, _ = O.brute_force(C)
    assert nbest == 1
    assert np.array_equal(_canon(lab), _canon(planted))
    assert bf == pytest.approx(-0.5 * np.linalg.slogdet(C)[1], rel=1e-12)


def test_brute_force_reports_the_tie_of_two_uncorrelated_singletons():
    """Two stocks with zero correlation to everything score the same apart or paired (c_s = n_s)."""
    C, planted = synth.block_correlation([3], [0.5], 2)
    bf, lab, nbest, _ = O.brute_force(C)
    assert nbest == 2
    assert bf == pytest.approx(-0.5 * np.linalg.slogdet(C)[1], rel=1e-12)


def test_brute_force_maximum_dominates_random_labelings():
    C, _ = _sample_corr(9, 60, seed=13)
    bf, lab, _, _ = O.brute_force(C)
    assert O.fitness(C, lab[None, :])[0] == bf
    pop = synth.random_labelings(500, 9, seed=14)
    assert np.all(O.fitness(C, pop) <= bf + 1e-12)
