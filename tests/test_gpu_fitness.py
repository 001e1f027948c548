"""GPU parity of pga_fitness (both forms), pga_correlate and pga_split against the CPU oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga, synth
from gpu_cases import bf16_emulated, corr, cs_bound_fp32, fitness_tol, l_bound_from_cs, say

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.fixture(autouse=True)
def _dense_route():
    """These tests check the O(N^2) pair-sum kernels: every individual takes that route
    (the cluster-pair route has its own tests)."""
    with pga.route(0.0):
        yield


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


FIT_CASES = [
    # N, P, K (labels drawn in [0, K)), seed
    (1, 3, 1, 0),
    (2, 5, 2, 1),
    (18, 100, 18, 2),
    (18, 100, 3, 3),
    (63, 70, 8, 4),
    (64, 64, 64, 5),
    (65, 129, 5, 6),
    (100, 200, 12, 7),
    (257, 65, 30, 8),
    (1024, 40, 40, 9),
    (1024, 33, 1024, 10),
]


@pytest.mark.parametrize("N,P,K,seed", FIT_CASES, ids=[f"N{c[0]}-P{c[1]}-K{c[2]}" for c in FIT_CASES])
def test_fitness_fp64_matches_oracle(N, P, K, seed):
    say(f"fitness fp64 N={N} P={P} K={K}")
    C, planted = corr(N, seed=seed)
    pop = synth.random_labelings(P, N, seed=seed, K=K)
    if P > 4:
        pop[-2:] = synth.perturbed_labelings(planted, 2, 0.05, seed)  # near-planted rows
    f_o, ns_o, cs_o, mag = O.fitness(C, pop, want_ns=True, want_cs=True, want_mag=True)
    st = pga.new_status()
    f_g, ns_g, cs_g = pga.fitness(_g(C), _g(pop), "fp64", want_ns=True, want_cs=True, status=st)
    torch.cuda.synchronize()
    assert np.array_equal(ns_g.cpu().numpy(), ns_o)
    assert np.all(np.abs(cs_g.cpu().numpy() - cs_o) <= 1e-11 * np.maximum(1.0, ns_o.astype(float) ** 2))
    d = np.abs(f_g.cpu().numpy() - f_o)
    assert np.all(d <= fitness_tol(mag)), float(np.max(d / np.maximum(mag, 1e-300)))
    assert st.cpu().numpy().sum() == 0


def test_fitness_planted_config3_shape():
    """N = 1024 with the 32-cluster geometric structure: near-planted labelings (converged-like)."""
    say("fitness fp64 config-3 shape")
    w = synth.config3(T=512)
    C = O.correlate(w.R)
    pop = synth.perturbed_labelings(w.planted, 24, 0.02, seed=3)
    pop[0] = w.planted
    f_o, mag = O.fitness(C, pop, want_mag=True)
    f_g = pga.fitness(_g(C), _g(pop), "fp64").cpu().numpy()
    assert np.all(np.abs(f_g - f_o) <= fitness_tol(mag))


def test_fitness_identity_is_exactly_zero():
    say("fitness C = I")
    for N in (1, 7, 64, 300):
        C = np.eye(N)
        pop = synth.random_labelings(17, N, seed=N, K=max(1, N // 4))
        for form in ("fp64", "bf16x2"):
            hi, lo = pga.split(_g(C)) if form == "bf16x2" else (None, None)
            f = pga.fitness(_g(C), _g(pop), form, hi=hi, lo=lo).cpu().numpy()
            assert np.all(f == 0.0), (N, form)


def test_fitness_errors_and_status_match_oracle():
    say("fitness invalid labels / domain")
    C = np.array([[1.0, 1.0, 0.1, 0.0], [1.0, 1.0, 0.1, 0.0], [0.1, 0.1, 1.0, -1.0], [0.0, 0.0, -1.0, 1.0]])
    pop = np.array([[0, 0, 1, 2],      # identical pair -> c = n^2 -> domain
                    [0, 1, 2, 2],      # anti-correlated pair -> c = 0 -> domain
                    [0, 1, 4, 3],      # label out of range
                    [-1, 0, 0, 0],     # negative label
                    [0, 1, 2, 3],      # singletons, fine
                    [1, 1, 1, 1]], dtype=np.int32)   # both bad clusters merged: c_s inside the domain
    st_o = O.status_zero()
    f_o, ns_o, cs_o = O.fitness(C, pop, want_ns=True, want_cs=True, status=st_o)
    for form in ("fp64", "bf16x2"):
        st = pga.new_status()
        hi, lo = pga.split(_g(C)) if form == "bf16x2" else (None, None)
        f_g, ns_g, cs_g = pga.fitness(_g(C), _g(pop), form, hi=hi, lo=lo, want_ns=True, want_cs=True, status=st)
        f_g = f_g.cpu().numpy()
        rtol, atol = (1e-12, 1e-13) if form == "fp64" else (1e-4, 1e-5)
        assert np.array_equal(np.isinf(f_g), np.isinf(f_o)), form
        assert np.allclose(f_g[np.isfinite(f_o)], f_o[np.isfinite(f_o)], rtol=rtol, atol=atol)
        assert np.array_equal(st.cpu().numpy(), st_o), form
        assert np.array_equal(ns_g.cpu().numpy(), ns_o)
        assert np.allclose(cs_g.cpu().numpy(), cs_o, rtol=rtol, atol=atol)


def test_fitness_empty_population_is_a_noop():
    C = _g(np.eye(5))
    f = pga.fitness(C, torch.empty((0, 5), dtype=torch.int32, device=DEV))
    assert f.numel() == 0


def test_fitness_maximum_n():
    N = pga.N_MAX
    say(f"fitness fp64 N_MAX={N}")
    C, _ = corr(N, T=64, seed=11)
    pop = synth.random_labelings(3, N, seed=12, K=200)
    f_o, mag = O.fitness(C, pop, want_mag=True)
    f_g = pga.fitness(_g(C), _g(pop), "fp64").cpu().numpy()
    assert np.all(np.abs(f_g - f_o) <= fitness_tol(mag))
    hi, lo = pga.split(_g(C))
    f_b = pga.fitness(_g(C), _g(pop), "bf16x2", hi=hi, lo=lo).cpu().numpy()
    assert np.all(np.abs(f_b - f_o) <= 1e-4 * mag + 1e-9)


def test_fitness_is_deterministic():
    C, _ = corr(300, seed=13)
    pop = _g(synth.random_labelings(200, 300, seed=14, K=20))
    Cg = _g(C)
    hi, lo = pga.split(Cg)
    for form in ("fp64", "bf16x2"):
        a = pga.fitness(Cg, pop, form, hi=hi, lo=lo)
        b = pga.fitness(Cg, pop, form, hi=hi, lo=lo)
        assert torch.equal(a, b)


# ---------------------------------------------------------------- correlation and split
CORR_CASES = [(1, 5), (2, 3), (18, 500), (70, 300), (100, 2000), (257, 130),
              # slices of the Gram's t range: several per tile, ragged last chunks, one slice
              (64, 390), (1024, 390), (130, 17), (513, 700), (4096, 40)]


@pytest.mark.parametrize("N,T", CORR_CASES, ids=[f"N{n}-T{t}" for n, t in CORR_CASES])
def test_correlate_matches_oracle(N, T):
    say(f"correlate N={N} T={T}")
    rng = np.random.default_rng(N * 7 + T)
    R = rng.standard_normal((N, T)) * rng.uniform(0.5, 3.0, size=(N, 1)) + rng.uniform(-2, 2, size=(N, 1))
    if N >= 3:
        R[1] = 0.25                       # a zero-variance stock
    st_o = O.status_zero()
    C_o = O.correlate(R, status=st_o)
    st = pga.new_status()
    C_g = pga.correlate(_g(R), status=st).cpu().numpy()
    assert np.max(np.abs(C_g - C_o)) <= 1e-12
    assert np.all(np.diag(C_g) == 1.0)
    assert np.array_equal(C_g, C_g.T)
    assert np.array_equal(st.cpu().numpy(), st_o)


def test_correlate_strided_rows():
    """Rows of R with a leading dimension larger than T (a window of a longer series)."""
    say("correlate strided rows")
    rng = np.random.default_rng(5)
    full = rng.standard_normal((300, 1000))
    R = full[:, 100:777]
    C_o = O.correlate(R)
    Rg = _g(full)[:, 100:777]
    assert Rg.stride(0) == 1000
    C_g = pga.correlate(Rg).cpu().numpy()
    assert np.max(np.abs(C_g - C_o)) <= 1e-12


def test_correlate_config3_shape_and_split():
    say("correlate config-3 shape")
    w = synth.config3(T=1024)
    C_o = O.correlate(w.R)
    C_g, _, _ = pga.correlate(_g(w.R), split=True)
    C_g = C_g.cpu().numpy()
    assert np.max(np.abs(C_g - C_o)) <= 1e-12
    hi, lo = pga.split(_g(C_o))              # the split of the oracle's matrix, bit for bit
    hi_o, lo_o = O.split_bf16(C_o)
    N = w.N
    h = hi.cpu().numpy().view(np.uint16)
    l = lo.cpu().numpy().view(np.uint16)
    assert np.array_equal(h[:N, :N], hi_o) and np.array_equal(l[:N, :N], lo_o)


def test_split_bit_exact_including_ties_and_padding():
    say("split special values")
    rng = np.random.default_rng(21)
    N = 45
    C = rng.uniform(-1, 1, size=(N, N))
    vals = [np.array([b | 0x8000], dtype=np.uint32).view(np.float32)[0] for b in
            (0x3F800000, 0x3F810000, 0xBE120000, 0x3C7F0000)]
    C.flat[:4] = vals
    C.flat[4:9] = [0.0, -0.0, 2.0**-130, -(2.0**-140), 1.0 - 2.0**-40]
    C.flat[9] = 3.0e-39
    hi_o, lo_o = O.split_bf16(C)
    hi, lo = pga.split(_g(C))
    ld = pga.split_ld(N)
    assert hi.shape == (ld, ld)
    h = hi.cpu().numpy().view(np.uint16)
    l = lo.cpu().numpy().view(np.uint16)
    assert np.array_equal(h[:N, :N], hi_o)
    assert np.array_equal(l[:N, :N], lo_o)
    assert not h[N:, :].any() and not h[:, N:].any() and not l[N:, :].any() and not l[:, N:].any()


# ---------------------------------------------------------------- BF16x2 MFMA form
BF_CASES = [(2, 4, 2, 0), (18, 100, 4, 1), (33, 40, 33, 2), (100, 64, 10, 3), (257, 40, 30, 4),
            (1024, 24, 40, 5), (1024, 17, 1024, 6)]


@pytest.mark.parametrize("N,P,K,seed", BF_CASES, ids=[f"N{c[0]}-P{c[1]}-K{c[2]}" for c in BF_CASES])
def test_fitness_bf16x2_matches_oracle_on_split_matrix(N, P, K, seed):
    """The MFMA form against the oracle run on hi + lo in FP64: only FP32 accumulation differs."""
    say(f"fitness bf16x2 N={N} P={P} K={K}")
    C, planted = corr(N, seed=100 + seed)
    pop = synth.random_labelings(P, N, seed=seed, K=K)
    pop[-1] = planted
    Cg = _g(C)
    hi, lo = pga.split(Cg)
    hi_n = hi.cpu().numpy().view(np.uint16)[:N, :N]
    lo_n = lo.cpu().numpy().view(np.uint16)[:N, :N]
    hi_o, lo_o = O.split_bf16(C)
    assert np.array_equal(hi_n, hi_o) and np.array_equal(lo_n, lo_o)
    Ce = bf16_emulated(C, hi_o, lo_o)
    f_e, ns_e, cs_e = O.fitness(Ce, pop, want_ns=True, want_cs=True)
    f_g, ns_g, cs_g = pga.fitness(Cg, _g(pop), "bf16x2", hi=hi, lo=lo, want_ns=True, want_cs=True)
    ns_g, cs_g, f_g = ns_g.cpu().numpy(), cs_g.cpu().numpy(), f_g.cpu().numpy()
    assert np.array_equal(ns_g, ns_e)
    bnd = cs_bound_fp32(Ce, pop)
    assert np.all(np.abs(cs_g - cs_e) <= bnd)
    assert np.all(np.abs(f_g - f_e) <= l_bound_from_cs(ns_e, cs_e, bnd))
    # and against the FP64 oracle on C itself: the split's own error, reported
    f_o, mag = O.fitness(C, pop, want_mag=True)
    rel = np.abs(f_g - f_o) / np.maximum(mag, 1e-300)
    say(f"  bf16x2 vs fp64 oracle: max |dL|/M = {rel.max():.3e}")
    assert rel.max() < 1e-4


@pytest.mark.parametrize("N,P", [(100, 40), (257, 19)], ids=["N100-P40", "N257-P19"])
def test_bf16x2_invalid_labels_do_not_disturb_other_individuals(N, P):
    """Individuals with labels outside [0, N) share workgroups with valid ones: they come out -inf
    (status counted as by the oracle), and every valid individual still matches the oracle, in
    every kernel variant (the pair-sum clamps labels for addressing only)."""
    say(f"bf16x2 invalid labels mixed N={N} P={P}")
    C, _ = corr(N, seed=40 + N)
    pop = synth.random_labelings(P, N, seed=N, K=max(2, N // 8))
    rng = np.random.default_rng(N)
    bad = rng.choice(P, size=P // 4, replace=False)
    for k, p in enumerate(bad):
        pop[p, rng.integers(0, N)] = (N + 3) if k % 2 == 0 else -7
    st_o = O.status_zero()
    f_o, ns_o, cs_o, mag = O.fitness(C, pop, want_ns=True, want_cs=True, want_mag=True, status=st_o)
    assert np.all(np.isinf(f_o[bad]))
    Cg = _g(C)
    hi, lo = pga.split(Cg)
    ok = np.isfinite(f_o)
    try:
        for v in range(len(pga.variants("bf16x2"))):
            pga.tune_set("bf16x2", N, P, v)
            st = pga.new_status()
            f_g, ns_g, cs_g = pga.fitness(Cg, _g(pop), "bf16x2", hi=hi, lo=lo, want_ns=True, want_cs=True, status=st)
            f_g, ns_g, cs_g = f_g.cpu().numpy(), ns_g.cpu().numpy(), cs_g.cpu().numpy()
            assert np.array_equal(np.isinf(f_g), ~ok), v
            assert np.array_equal(st.cpu().numpy(), st_o), v
            assert np.array_equal(ns_g, ns_o), v                     # zeros for the invalid individuals
            assert np.all(cs_g[~ok] == 0.0), v
            assert np.all(np.abs(f_g[ok] - f_o[ok]) <= 1e-4 * mag[ok] + 1e-9), v
    finally:
        pga.tune_set("bf16x2", N, P, -1)
