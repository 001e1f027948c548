"""Pins for the oracle's correlation (Eq. 7), BF16 split and Philox4x32-10."""
import os

import numpy as np
import pytest

import oracle as O
from paper_1403_4099_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- correlation
@pytest.mark.parametrize("cfg", ["c1", "c2"])
def test_correlate_matches_numpy_corrcoef(cfg):
    w = synth.config1() if cfg == "c1" else synth.config2()
    C = O.correlate(w.R)
    ref = np.corrcoef(w.R)
    assert np.max(np.abs(C - ref)) < 1e-12
    assert np.all(np.diag(C) == 1.0)
    assert np.array_equal(C, C.T)
    assert np.all(np.abs(C) <= 1.0)


def test_correlate_affine_invariance():
    rng = np.random.default_rng(3)
    R = rng.standard_normal((12, 80))
    a = rng.uniform(0.1, 10.0, size=(12, 1))
    b = rng.uniform(-5.0, 5.0, size=(12, 1))
    sgn = np.where(rng.random((12, 1)) < 0.3, -1.0, 1.0)
    C = O.correlate(R)
    C2 = O.correlate(sgn * a * R + b)
    assert np.max(np.abs(C2 - C * (sgn @ sgn.T))) < 1e-12


def test_correlate_zero_variance_and_clamp():
    rng = np.random.default_rng(4)
    R = rng.standard_normal((5, 40))
    R[2] = 3.25                      # constant row
    R[4] = R[0] * 2.0 + 1.0          # perfectly correlated with row 0
    st = O.status_zero()
    C = O.correlate(R, status=st)
    assert st[2] == 1
    assert C[2, 2] == 1.0
    assert np.all(C[2, [0, 1, 3, 4]] == 0.0) and np.all(C[[0, 1, 3, 4], 2] == 0.0)
    assert C[0, 4] == pytest.approx(1.0, abs=1e-15) and C[0, 4] <= 1.0


# ---------------------------------------------------------------- BF16 split
def _bf16_neighbours(x):
    """The two bfloat16 values bracketing x, by truncating the float32 pattern (exact for |x| in float32 range)."""
    f = np.float32(x)
    assert float(f) == x, "test values must be float32-exact"
    u = np.array([f]).view(np.uint32)[0]
    lo_bits = np.uint32(u & 0xFFFF0000)
    hi_bits = np.uint32(lo_bits + 0x10000)
    to = lambda b: float(np.array([b], dtype=np.uint32).view(np.float32)[0])
    return to(lo_bits), to(hi_bits), int(lo_bits >> 16)


def test_split_is_round_to_nearest_even():
    rng = np.random.default_rng(5)
    xs = list(np.float32(rng.uniform(-1, 1, 2000)).astype(np.float64))
    # exact ties between neighbours: mantissa bit pattern ...1000 0000 0000 0000 in the low half
    for base in (0x3F800000, 0x3F810000, 0xBE120000, 0x3C7F0000):
        t = np.array([base | 0x8000], dtype=np.uint32).view(np.float32)[0]
        xs.append(float(t))
    xs += [0.0, 1.0, -1.0, 2.0**-130, -(2.0**-140)]
    xs = np.array(xs)
    hi, lo = O.split_bf16(xs)
    hv = O.bf16_to_f64(hi)
    for x, h, hb in zip(xs, hv, hi):
        a, b, abits = _bf16_neighbours(x)
        da, db = abs(x - a), abs(x - b)
        if da < db:
            assert h == a
        elif db < da:
            assert h == b
        else:   # tie: even mantissa
            assert (int(hb) & 1) == 0 and h in (a, b)


def test_split_residual_bound_and_exact_values():
    rng = np.random.default_rng(6)
    C = rng.uniform(-1, 1, size=5000)
    hi, lo = O.split_bf16(C)
    h, l = O.bf16_to_f64(hi), O.bf16_to_f64(lo)
    # |C - hi| <= 2^-8 |C|, |C - hi - lo| <= 2^-16 |C| (8 significant bits each)
    assert np.all(np.abs(C - h) <= 2.0**-8 * np.abs(C))
    assert np.all(np.abs(C - h - l) <= 2.0**-16 * np.abs(C))
    hi, lo = O.split_bf16(np.array([1.0, -1.0, 0.0, 0.5]))
    assert list(hi) == [0x3F80, 0xBF80, 0x0000, 0x3F00]
    assert list(lo) == [0, 0, 0, 0]


# ---------------------------------------------------------------- Philox
def test_philox_known_answer_vectors():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(x, 16) for x in line.split()])
    assert len(rows) == 3
    for r in rows:
        out = O.philox(r[0:4], r[4:6])
        assert list(out) == r[6:10]


def test_init_population_uniform_and_in_range():
    N, P = 37, 4000
    pop = O.init_pop(N, P, seed=12345, inst=3, gen0=7)
    assert pop.min() >= 0 and pop.max() < N
    counts = np.bincount(pop.ravel(), minlength=N)
    expect = P * N / N
    chi2 = float(np.sum((counts - expect) ** 2 / expect))
    # chi-square with 36 dof: mean 36, sd 8.5; 6 sd bound
    assert chi2 < 36 + 6 * 8.5
    # different instance id, generation or seed changes the stream
    assert not np.array_equal(pop, O.init_pop(N, P, seed=12345, inst=4, gen0=7))
    assert not np.array_equal(pop, O.init_pop(N, P, seed=12345, inst=3, gen0=8))
    assert not np.array_equal(pop, O.init_pop(N, P, seed=12346, inst=3, gen0=7))
