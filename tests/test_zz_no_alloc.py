"""pga_fitness_noalloc (scratch in the library's static device array) against
pga_fitness (caller workspace), through the C ABI: two calls in a row, the
second smaller, in both forms, with and without the cluster-pair route. Both
entry points run the same kernels on the same inputs, so fitness, n_s and c_s
must agree bit for bit; the first call is also held to the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1403_4099_amd import pga, synth
from gpu_cases import corr, fitness_tol, say

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _pop(N, P, K, seed, planted):
    pop = synth.random_labelings(P, N, seed=seed, K=K)
    pop[-3:] = synth.perturbed_labelings(planted, 3, 0.05, seed)
    return pop


def _both(C, pop, form, hi, lo):
    st_w, st_n = pga.new_status(), pga.new_status()
    f_w, ns_w, cs_w = pga.fitness(C, pop, form, hi=hi, lo=lo, want_ns=True, want_cs=True, status=st_w)
    f_n, ns_n, cs_n = pga.fitness_noalloc(C, pop, form, hi=hi, lo=lo, want_ns=True, want_cs=True, status=st_n)
    torch.cuda.synchronize()
    return ((f_w.cpu().numpy(), ns_w.cpu().numpy(), cs_w.cpu().numpy(), st_w.cpu().numpy()),
            (f_n.cpu().numpy(), ns_n.cpu().numpy(), cs_n.cpu().numpy(), st_n.cpu().numpy()))


@pytest.mark.parametrize("route", [0.0, 1.0 / 64.0, 1.0], ids=["pairsum", "default", "cluster-pairs"])
@pytest.mark.parametrize("form", ["fp64", "bf16x2"])
def test_noalloc_equals_workspace_entry(form, route):
    # first call: several pair-sum tiles and a ragged tail; second call: smaller
    for k, (N, P, K, seed) in enumerate([(300, 200, 40, 11), (70, 33, 12, 12)]):
        say(f"noalloc {form} route={route} call {k}: N={N} P={P}")
        C_np, planted = corr(N, seed=seed)
        pop_np = _pop(N, P, K, seed, planted)
        C, pop = _g(C_np), _g(pop_np)
        hi, lo = pga.split(C) if form == "bf16x2" else (None, None)
        with pga.route(route):
            (f_w, ns_w, cs_w, st_w), (f_n, ns_n, cs_n, st_n) = _both(C, pop, form, hi, lo)
        assert np.array_equal(f_n.view(np.int64), f_w.view(np.int64))
        assert np.array_equal(ns_n, ns_w)
        assert np.array_equal(cs_n.view(np.int64), cs_w.view(np.int64))
        assert np.array_equal(st_n, st_w) and st_n.sum() == 0
        if form == "fp64" and k == 0:
            f_o, mag = O.fitness(C_np, pop_np, want_mag=True)
            assert np.all(np.abs(f_n - f_o) <= fitness_tol(mag))


def test_noalloc_benchmark_size_fits():
    """N = 1024, P = 4096 (the benchmark's fitness call) fits the static scratch in both forms,
    followed by a much smaller call: both equal the workspace entry point bit for bit."""
    for N, P in ((1024, 4096), (40, 9)):
        say(f"noalloc full-size sequence N={N} P={P}")
        C_np, planted = corr(N, seed=21)
        pop_np = _pop(N, P, max(2, N // 3), 21, planted)
        C, pop = _g(C_np), _g(pop_np)
        hi, lo = pga.split(C)
        for form in ("bf16x2", "fp64"):
            assert pga.fitness_ws_bytes(N, P, form) <= pga.noalloc_max_bytes()
            (f_w, ns_w, cs_w, _), (f_n, ns_n, cs_n, _) = _both(C, pop, form, hi, lo)
            assert np.array_equal(f_n.view(np.int64), f_w.view(np.int64))
            assert np.array_equal(ns_n, ns_w)
            assert np.array_equal(cs_n.view(np.int64), cs_w.view(np.int64))


def test_noalloc_rejects_oversize_before_any_work():
    N, P = 2048, 4096
    assert pga.fitness_ws_bytes(N, P, "fp64") > pga.noalloc_max_bytes()
    C = torch.zeros((N, N), dtype=torch.float64, device=DEV)
    pop = torch.zeros((P, N), dtype=torch.int32, device=DEV)
    f = torch.full((P,), 7.0, dtype=torch.float64, device=DEV)
    with pytest.raises(pga.PgaError, match="size beyond"):
        pga.fitness_noalloc(C, pop, "fp64", out=f)
    torch.cuda.synchronize()
    assert bool((f == 7.0).all())
