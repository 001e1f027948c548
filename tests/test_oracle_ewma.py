"""Oracle pins for the online EWMA correlation (Section 4.2.5 pre-processing:
market mode removed, exponentially weighted covariance, its correlation).

Pins: closed forms for one observation and for lambda = 0, the zero column sums
that removing the market return forces, continuation across calls, and the
weighted Gram matrix computed independently by numpy."""
import numpy as np
import pytest

from oracle import oracle as O


def _R(N, T, seed=0):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(T)
    return 0.4 * f[None, :] + rng.standard_normal((N, T))


def test_single_observation_gives_signs():
    R = _R(7, 1)
    for market in (False, True):
        C, S = O.ewma(R, 0.98, market=market)
        x = R[:, 0] - (R[:, 0].mean() if market else 0.0)
        assert np.array_equal(np.sign(C), np.where(np.eye(7, dtype=bool), 1.0, np.sign(np.outer(x, x))))
        assert np.allclose(np.abs(C), 1.0, rtol=0, atol=4e-16) and np.all(np.diag(C) == 1.0)
        assert np.allclose(S, 0.02 * np.outer(x, x), rtol=1e-14, atol=0)


def test_lambda_zero_keeps_only_the_last_observation():
    R = _R(6, 40, 1)
    C, S = O.ewma(R, 0.0, market=False)
    x = R[:, -1]
    assert np.array_equal(S, np.outer(x, x))
    assert np.allclose(np.abs(C), 1.0, rtol=0, atol=4e-16)


def test_market_removal_zeroes_column_sums():
    R = _R(12, 300, 2)
    _, S = O.ewma(R, 0.98, market=True)
    assert np.all(np.abs(S.sum(axis=0)) <= 1e-13 * np.abs(S).max())
    _, S2 = O.ewma(R, 0.98, market=False)
    assert np.abs(S2.sum(axis=0)).max() > 1e-3


@pytest.mark.parametrize("lam,market", [(0.98, True), (0.9, False), (0.5, True)])
def test_weighted_gram_matches_numpy(lam, market):
    N, T = 9, 200
    R = _R(N, T, 3)
    C, S = O.ewma(R, lam, market=market)
    X = R - (R.mean(axis=0, keepdims=True) if market else 0.0)
    w = (1 - lam) * lam ** np.arange(T - 1, -1, -1)
    S_np = (X * w[None, :]) @ X.T
    assert np.allclose(S, S_np, rtol=1e-12, atol=1e-15)
    d = np.sqrt(np.diag(S_np))
    C_np = np.clip(S_np / np.outer(d, d), -1, 1)
    np.fill_diagonal(C_np, 1.0)
    assert np.allclose(C, C_np, rtol=1e-12, atol=1e-14)


def test_two_calls_continue_the_recursion():
    R = _R(8, 150, 4)
    C, S = O.ewma(R, 0.97)
    C1, S1 = O.ewma(R[:, :60], 0.97)
    C2, S2 = O.ewma(R[:, 60:], 0.97, S=S1)
    assert np.array_equal(S2, S) and np.array_equal(C2, C)


def test_zero_variance_stock_is_counted_and_zeroed():
    R = _R(5, 50, 5)
    R[2] = 0.0                                   # a stock that never moves (no market step)
    st = O.status_zero()
    C, S = O.ewma(R, 0.98, market=False, status=st)
    assert st[2] == 1 and np.all(C[2, [0, 1, 3, 4]] == 0) and C[2, 2] == 1
