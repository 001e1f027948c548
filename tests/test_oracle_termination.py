"""Oracle pins for the GA termination test (Algorithm 1, "determine if termination
criteria are met"; Table 3: error tolerance, stall generations).

The pins tie the terminating run to the plain run (which the GA tests already pin)
and to cases whose stop point is fixed by the definition alone."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1403_4099_amd import synth


@pytest.fixture(scope="module")
def c1():
    w = synth.config1()
    return O.correlate(w.R)


def test_disabled_equals_plain_evolve(c1):
    p1, f1, s1 = O.evolve(c1, 64, 25, seed=3)
    p2, f2, s2, st = O.evolve_term(c1, 64, 25, 0, 1e-5, seed=3)
    assert np.array_equal(p1, p2) and np.array_equal(f1, f2) and np.array_equal(s1, s2)
    assert st[2] == 0 and st[3] == 25


def test_huge_tolerance_stops_after_exactly_stall_generations(c1):
    # No generation after the first can improve, so the stall count reaches k at
    # generation k: k generations are bred and k + 1 statistics rows written.
    for k in (1, 4, 9):
        _, _, st, state = O.evolve_term(c1, 40, 50, k, 1e9, seed=1)
        assert state[2] == 1 and state[3] == k and state[1] == k
        assert np.isfinite(st[: k + 1, 0]).all() and np.isnan(st[k + 1:, 0]).all()


def test_negative_tolerance_never_stops_with_elitism(c1):
    # With elites the best fitness never falls, so b > ref - |tol| max(1, |ref|) always holds.
    _, _, st, state = O.evolve_term(c1, 40, 30, 2, -0.5, E=2, seed=2)
    assert state[2] == 0 and state[3] == 30 and np.isfinite(st[:, 0]).all()


def test_stopped_run_is_the_plain_run_cut_at_the_stop(c1):
    pop, fit, st, state = O.evolve_term(c1, 100, 400, 20, 1e-5, seed=0)
    assert state[2] == 1
    g = int(state[3])
    assert 20 <= g < 400
    p2, f2, s2 = O.evolve(c1, 100, g, seed=0)
    assert np.array_equal(pop, p2) and np.array_equal(fit, f2)
    assert np.array_equal(st[: g + 1], s2)
    # the last 20 evaluated generations did not improve on the reference by the tolerance
    best = st[: g + 1, 0]
    assert best[g] <= state[0] + 1e-5 * max(1.0, abs(state[0]))


def test_continuation_matches_one_call(c1):
    pop, fit, st, state = O.evolve_term(c1, 60, 300, 15, 1e-5, seed=5)
    g = int(state[3])
    assert state[2] == 1 and g > 12
    # same run in two calls: the second continues from the first call's state and generation
    pa, _, sa, sta = O.evolve_term(c1, 60, 12, 15, 1e-5, seed=5)
    assert sta[2] == 0 and sta[3] == 12
    pb, fb, sb, stb = O.evolve_term(c1, 60, 300, 15, 1e-5, seed=5, pop=pa, state=sta, gen0=12)
    assert np.array_equal(stb, state) and np.array_equal(pb, pop) and np.array_equal(fb, fit)
    # the second call's rows are the one-call rows from generation 12 on (its row 0 re-evaluates
    # generation 12, which the first call already recorded as its last row)
    assert np.array_equal(sb[: g - 12 + 1], st[12: g + 1])
    assert np.array_equal(sa[12], st[12])


@pytest.mark.parametrize("chunk", [1, 3, 7, 12])
def test_any_split_into_calls_equals_one_call(c1, chunk):
    # Algorithm 1 tests each generation once: a continuing call re-evaluates the population the
    # previous call tested last and must not test it again, so a run cut into calls of `chunk`
    # generations stops at the same generation with the same state and population as one call.
    pop, fit, _, state = O.evolve_term(c1, 60, 300, 15, 1e-5, seed=5)
    assert state[2] == 1
    p, s, g0 = None, None, 0
    for _ in range(400):
        p, f, _, s = O.evolve_term(c1, 60, chunk, 15, 1e-5, seed=5, pop=p, state=s, gen0=g0)
        g0 = int(s[3])
        if s[2] == 1:
            break
    assert np.array_equal(s, state) and np.array_equal(p, pop) and np.array_equal(f, fit)


def test_call_after_stop_changes_nothing(c1):
    pop, fit, _, state = O.evolve_term(c1, 50, 200, 5, 1e9, seed=4)
    assert state[2] == 1
    p2, f2, s2, st2 = O.evolve_term(c1, 50, 30, 5, 1e9, seed=4, pop=pop, state=state, gen0=int(state[3]))
    assert np.array_equal(p2, pop) and np.array_equal(f2, fit) and np.array_equal(st2, state)
    assert np.isnan(s2).all()


def test_stops_at_the_brute_force_optimum():
    # Small planted problem: the GA reaches the exact optimum (brute force over all
    # set partitions) and then stalls, so the terminating run ends early with it.
    rng = np.random.default_rng(11)
    R = synth.one_factor_returns([4, 3, 2], rng.uniform(0.5, 0.8, 3), 0, 400, rng, shuffle=True)[0]
    C = O.correlate(R)
    bf, _, _, _ = O.brute_force(C)
    pop, fit, st, state = O.evolve_term(C, 64, 600, 40, 1e-9, seed=0)
    assert state[2] == 1 and state[3] < 600
    assert abs(fit.max() - bf) <= 1e-12 * max(1.0, abs(bf))
