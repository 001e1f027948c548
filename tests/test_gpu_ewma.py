"""GPU parity of the online EWMA correlation (pga_ewma) against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga
from gpu_cases import say

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _R(N, T, seed=0):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal(T)
    return 0.4 * f[None, :] + rng.standard_normal((N, T))


CASES = [(1, 10, 0.98, True), (7, 1, 0.98, True), (64, 390, 0.98, True), (100, 500, 0.9, False),
         (130, 77, 0.0, True), (300, 390, 0.98, True)]


@pytest.mark.parametrize("N,T,lam,market", CASES, ids=[f"N{c[0]}-T{c[1]}-l{c[2]}-m{int(c[3])}" for c in CASES])
def test_ewma_matches_oracle(N, T, lam, market):
    say(f"ewma N={N} T={T} lam={lam} market={market}")
    R = _R(N, T, N + T)
    C_o, S_o = O.ewma(R, lam, market=market)
    S = torch.full((N, N), float("nan"), dtype=torch.float64, device=DEV)   # ignored with reset
    st = pga.new_status()
    C, hi, lo = pga.ewma(torch.from_numpy(R).to(DEV), S, lam, reset=True, market=market, split=True, status=st)
    Sg, Cg = S.cpu().numpy(), C.cpu().numpy()
    assert np.allclose(Sg, S_o, rtol=1e-11, atol=1e-13 * np.abs(S_o).max())
    assert np.allclose(Cg, C_o, rtol=0, atol=1e-11)
    assert np.array_equal(np.diag(Cg), np.ones(N)) and np.array_equal(Cg, Cg.T)
    h_o, l_o = O.split_bf16(Cg)
    ld = pga.split_ld(N)
    assert np.array_equal(hi.cpu().numpy().view(np.uint16)[:N, :N], h_o)
    assert np.array_equal(lo.cpu().numpy().view(np.uint16)[:N, :N], l_o)
    assert int(st[2]) == int((np.diag(S_o) == 0).sum())


def test_ewma_continuation_and_zero_variance():
    say("ewma continuation")
    N, T = 90, 400
    R = _R(N, T, 9)
    R[5] = 0.0                                   # zero variance without the market step
    C_o, S_o = O.ewma(R, 0.98, market=False)
    Rg = torch.from_numpy(R).to(DEV)
    S = torch.zeros((N, N), dtype=torch.float64, device=DEV)
    pga.ewma(Rg[:, :150].contiguous(), S, 0.98, reset=True, market=False)
    st = pga.new_status()
    C = pga.ewma(Rg[:, 150:].contiguous(), S, 0.98, reset=False, market=False, status=st)
    assert np.allclose(S.cpu().numpy(), S_o, rtol=1e-11, atol=1e-13 * np.abs(S_o).max())
    assert np.allclose(C.cpu().numpy(), C_o, rtol=0, atol=1e-11)
    assert int(st[2]) == 1


def test_ewma_argument_errors():
    R = torch.zeros((4, 8), dtype=torch.float64, device=DEV)
    S = torch.zeros((4, 4), dtype=torch.float64, device=DEV)
    with pytest.raises(pga.PgaError):
        pga.ewma(R, S, 1.0)
    with pytest.raises(pga.PgaError):
        pga.ewma(R, S, -0.1)
