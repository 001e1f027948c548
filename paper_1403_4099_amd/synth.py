"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only draws inputs. It holds none of the method's arithmetic: no
correlation, no likelihood, no genetic operator. Every function is a pure
function of its seed (numpy PCG64), so the CPU oracle and the HIP path see
bit-identical inputs.

Returns follow the one-factor-per-cluster model of the paper's Section 2.2.3
(Eq. 2) in the parameterisation r_it = sqrt(g_s) f_st + sqrt(1 - g_s) e_it,
f and e iid N(0,1), so two stocks of cluster s have population correlation
g_s. Stocks outside every planted cluster are pure noise (g = 0). Stock order
is shuffled so planted clusters are not contiguous index ranges.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Workload:
    """One correlation window: returns R (N x T, float64) and its planted partition."""

    name: str
    R: np.ndarray                # (N, T) float64, row-major
    planted: np.ndarray          # (N,) int32, planted cluster id per stock; noise stocks get unique ids
    sizes: list = field(default_factory=list)   # planted cluster sizes (>= 2), before shuffling
    g: np.ndarray = None         # per planted cluster loading
    # GA settings that go with the workload
    P: int = 0
    G: int = 0
    elites: int = 2
    seed: int = 0                # Philox key for the GA

    @property
    def N(self) -> int:
        return self.R.shape[0]

    @property
    def T(self) -> int:
        return self.R.shape[1]


def one_factor_returns(sizes, g, n_noise, T, rng, shuffle=True):
    """Draw R for planted clusters `sizes` with loadings `g` plus `n_noise` noise stocks.

    Returns (R, planted) with planted labels: cluster k -> k, noise stock m ->
    len(sizes) + m (each noise stock is its own singleton).
    """
    sizes = [int(s) for s in sizes]
    N = sum(sizes) + int(n_noise)
    R = np.empty((N, T), dtype=np.float64)
    planted = np.empty(N, dtype=np.int32)
    row = 0
    for k, (n, gk) in enumerate(zip(sizes, g)):
        f = rng.standard_normal(T)
        e = rng.standard_normal((n, T))
        R[row:row + n] = np.sqrt(gk) * f[None, :] + np.sqrt(1.0 - gk) * e
        planted[row:row + n] = k
        row += n
    for m in range(int(n_noise)):
        R[row] = rng.standard_normal(T)
        planted[row] = len(sizes) + m
        row += 1
    if shuffle:
        perm = rng.permutation(N)
        R = R[perm]
        planted = planted[perm]
    return np.ascontiguousarray(R), np.ascontiguousarray(planted)


def _dirichlet_sizes(rng, k, total, minimum=2):
    """k sizes >= minimum summing to `total`: minimum each plus a largest-remainder split of the rest by Dir(1)."""
    p = rng.dirichlet(np.ones(k))
    extra = total - minimum * k
    raw = p * extra
    base = np.floor(raw).astype(np.int64)
    rem = extra - int(base.sum())
    order = np.argsort(-(raw - base), kind="stable")
    base[order[:rem]] += 1
    return [int(minimum + b) for b in base]


def config1(seed: int = 0) -> Workload:
    """N=18, T=500, planted 8/6/4, g ~ U[0.3,0.7]; P=100, G=200, 2 elites, Philox seed 0."""
    rng = np.random.default_rng(seed)
    sizes = [8, 6, 4]
    g = rng.uniform(0.3, 0.7, size=3)
    R, planted = one_factor_returns(sizes, g, 0, 500, rng)
    return Workload("plain-fp64-tiny N=18 T=500", R, planted, sizes, g, P=100, G=200, elites=2, seed=0)


def config2(seed: int = 1) -> Workload:
    """N=100, T=2000, 8 Dirichlet(1) clusters (min 2) over 90 stocks + 10 noise; g ~ U[0.2,0.8]; P=1024, G=500."""
    rng = np.random.default_rng(seed)
    sizes = _dirichlet_sizes(rng, 8, 90)
    g = rng.uniform(0.2, 0.8, size=8)
    R, planted = one_factor_returns(sizes, g, 10, 2000, rng)
    return Workload("plain-fp64-medium N=100 T=2000", R, planted, sizes, g, P=1024, G=500, elites=2, seed=0)


def geometric_sizes(rng, k, mean, N):
    """k sizes max(2, Geom(1/mean)); redraw the whole set while the sum exceeds N."""
    while True:
        s = np.maximum(2, rng.geometric(1.0 / mean, size=k))
        if int(s.sum()) <= N:
            return [int(x) for x in s]


def config3(seed: int = 2, N: int = 1024, T: int = 4096) -> Workload:
    """N=1024, T=4096, 32 clusters with sizes max(2, Geom(mean 28)), rest noise; g ~ U[0.1,0.6]; P=4096, G=300."""
    rng = np.random.default_rng(seed)
    sizes = geometric_sizes(rng, 32, 28.0, N)
    g = rng.uniform(0.1, 0.6, size=32)
    R, planted = one_factor_returns(sizes, g, N - sum(sizes), T, rng)
    return Workload(f"precision-form N={N} T={T}", R, planted, sizes, g, P=4096, G=300, elites=2, seed=0)


def config4_instance(i: int, T: int = 1024) -> Workload:
    """Instance i of the batched form: N ~ U{32..512}, k ~ U{2..12} Dir(1) clusters over floor(0.9N), g ~ U[0.2,0.7]."""
    rng = np.random.default_rng(3 + i)
    N = int(rng.integers(32, 513))
    k = int(rng.integers(2, 13))
    covered = int(np.floor(0.9 * N))
    sizes = _dirichlet_sizes(rng, k, covered)
    g = rng.uniform(0.2, 0.7, size=k)
    R, planted = one_factor_returns(sizes, g, N - covered, T, rng)
    return Workload(f"batched-instance-{i} N={N}", R, planted, sizes, g, P=512, G=200, elites=2, seed=0)


def random_labelings(P: int, N: int, seed: int, K: int | None = None) -> np.ndarray:
    """P uniform labelings with labels in [0, K) (K defaults to N), int32 (P, N)."""
    rng = np.random.default_rng(seed)
    K = N if K is None else K
    return rng.integers(0, K, size=(P, N), dtype=np.int64).astype(np.int32)


def perturbed_labelings(base: np.ndarray, P: int, frac: float, seed: int) -> np.ndarray:
    """P copies of `base` with about `frac` of the stocks moved to a uniformly drawn label in [0, N)."""
    rng = np.random.default_rng(seed)
    N = base.shape[0]
    out = np.repeat(base[None, :].astype(np.int32), P, axis=0)
    mask = rng.random((P, N)) < frac
    out[mask] = rng.integers(0, N, size=int(mask.sum()))
    return out


def block_correlation(sizes, rhos, n_single=0) -> tuple[np.ndarray, np.ndarray]:
    """Exact compound-symmetric block matrix: rho_s inside planted block s, 0 across, 1 on the diagonal.

    Blocks are contiguous (no shuffling) followed by `n_single` singletons.
    Returns (C, planted) with planted labels 0..len(sizes)-1 then singleton ids.
    """
    N = int(sum(sizes)) + int(n_single)
    C = np.zeros((N, N), dtype=np.float64)
    planted = np.empty(N, dtype=np.int32)
    row = 0
    for k, (n, r) in enumerate(zip(sizes, rhos)):
        C[row:row + n, row:row + n] = r
        planted[row:row + n] = k
        row += n
    for m in range(int(n_single)):
        planted[row] = len(sizes) + m
        row += 1
    np.fill_diagonal(C, 1.0)
    return C, planted


def random_symmetric_unit_diag(N: int, seed: int, scale: float = 0.3) -> np.ndarray:
    """A symmetric matrix with unit diagonal and off-diagonal entries U[-scale, scale] (not necessarily PSD)."""
    rng = np.random.default_rng(seed)
    A = rng.uniform(-scale, scale, size=(N, N))
    C = np.triu(A, 1)
    C = C + C.T
    np.fill_diagonal(C, 1.0)
    return C


# ---------------------------------------------------------------- serving stream
@dataclass
class Universe:
    uid: int
    N: int
    planted: np.ndarray      # current planted cluster id per stock
    g: np.ndarray            # loading per planted cluster


def serving_universes(seed: int = 4, counts=((64, 8), (256, 5), (1024, 3))):
    """Resident stock universes: 8 of 64 stocks, 5 of 256, 3 of 1024 (16 in all).

    Each has N // 16 planted clusters (at least 2) over 90% of its stocks, sizes by
    Dirichlet(1) (minimum 2), loadings g ~ U[0.2, 0.7]; the rest are noise stocks.
    """
    rng = np.random.default_rng(seed)
    us = []
    uid = 0
    for N, cnt in counts:
        for _ in range(cnt):
            k = max(2, N // 16)
            covered = int(0.9 * N)
            sizes = _dirichlet_sizes(rng, k, covered)
            planted = np.concatenate([np.repeat(np.arange(k), sizes), k + np.arange(N - covered)])
            planted = rng.permutation(planted).astype(np.int32)
            us.append(Universe(uid, N, planted, rng.uniform(0.2, 0.7, size=k)))
            uid += 1
    return us


def serving_stream(duration: float, rate: float = 200.0, T: int = 390, seed: int = 4,
                   ratio=(6, 3, 1), drift: float = 0.05):
    """Poisson arrivals over `duration` seconds; N-class drawn 6:3:1 over {64, 256, 1024},
    universe uniform within its class; before each window 5% of the universe's stocks move
    to another existing planted cluster; each window holds T fresh one-factor returns.

    Returns (universes, requests) with requests = [(arrival_s, uid, R (N x T float64))].
    """
    rng = np.random.default_rng(seed + 1)
    us = serving_universes(seed)
    by_n = {}
    for u in us:
        by_n.setdefault(u.N, []).append(u)
    classes = sorted(by_n)
    p = np.array(ratio, dtype=np.float64)
    p /= p.sum()
    out = []
    t = 0.0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        N = classes[int(rng.choice(len(classes), p=p))]
        u = by_n[N][int(rng.integers(len(by_n[N])))]
        k = len(u.g)
        moved = rng.random(N) < drift
        clustered = u.planted < k
        idx = np.nonzero(moved & clustered)[0]
        if idx.size:
            u.planted[idx] = rng.integers(0, k, size=idx.size)
        R = np.empty((N, T))
        f = rng.standard_normal((k, T))
        e = rng.standard_normal((N, T))
        lab = u.planted
        inc = lab < k
        gl = np.where(inc, u.g[np.minimum(lab, k - 1)], 0.0)
        R[:] = np.sqrt(gl)[:, None] * np.where(inc[:, None], f[np.minimum(lab, k - 1)], 0.0) \
            + np.sqrt(1.0 - gl)[:, None] * e
        out.append((t, u.uid, R))
    return us, out
