"""ctypes wrapper around oracle.c (plain FP64 CPU oracle; test infrastructure only).

The shared object is built with gcc at -O2 and no fast-math; `build()`
compiles it, `lib()` loads the built copy and builds it only when none exists.
"""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_OUT_DIR = os.path.join(_HERE, "_build")
_SO = os.path.join(_OUT_DIR, "liboracle.so")

P_CROSS_DEFAULT = int(0.9 * 2**32)      # crossover probability 0.9 (Table 3)

_lib = None


def build() -> str:
    os.makedirs(_OUT_DIR, exist_ok=True)
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ct.CDLL(_SO)
        d, i32, u32, u64, lng = ct.c_double, ct.c_int32, ct.c_uint32, ct.c_uint64, ct.c_long
        vp = ct.c_void_p
        L.oracle_correlate.argtypes = [vp, ct.c_int, ct.c_int, lng, vp, vp]
        L.oracle_correlate.restype = ct.c_int
        L.oracle_fitness_one.argtypes = [vp, ct.c_int, vp, vp, vp, vp, vp]
        L.oracle_fitness_one.restype = d
        L.oracle_fitness.argtypes = [vp, ct.c_int, vp, ct.c_int, vp, vp, vp, vp, vp]
        L.oracle_fitness.restype = None
        L.oracle_split_bf16.argtypes = [vp, lng, vp, vp]
        L.oracle_split_bf16.restype = None
        L.oracle_philox4x32_10.argtypes = [vp, vp, vp]
        L.oracle_philox4x32_10.restype = None
        L.oracle_init_pop.argtypes = [ct.c_int, ct.c_int, u64, u32, u32, vp]
        L.oracle_init_pop.restype = None
        L.oracle_rank.argtypes = [vp, ct.c_int, vp]
        L.oracle_rank.restype = None
        L.oracle_breed.argtypes = [vp, vp, ct.c_int, ct.c_int, ct.c_int, u32, u32, u64, u32, u32, vp]
        L.oracle_breed.restype = None
        L.oracle_stats.argtypes = [vp, ct.c_int, vp]
        L.oracle_stats.restype = None
        L.oracle_evolve.argtypes = [vp, ct.c_int, ct.c_int, ct.c_int, u32, u32, u64, u32, u32,
                                    ct.c_int, ct.c_int, vp, vp, vp, vp]
        L.oracle_evolve.restype = ct.c_int
        L.oracle_evolve_term.argtypes = [vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, u32, u32, u64, u32, u32,
                                         ct.c_int, ct.c_int, ct.c_int, d, vp, vp, vp, vp, vp]
        L.oracle_breed_sel.argtypes = [vp, vp, ct.c_int, ct.c_int, ct.c_int, ct.c_int, u32, u32, u64, u32,
                                       u32, vp]
        L.oracle_breed_sel.restype = None
        L.oracle_sus_parents.argtypes = [vp, ct.c_int, ct.c_int, u64, u32, u32, vp]
        L.oracle_sus_parents.restype = None
        L.oracle_shuffle_index.argtypes = [u32, u32, u64, u32, u32]
        L.oracle_shuffle_index.restype = u32
        L.oracle_ewma.argtypes = [vp, ct.c_int, ct.c_int, ct.c_long, d, ct.c_int, ct.c_int, vp, vp, vp]
        L.oracle_ewma.restype = None
        L.oracle_evolve_term.restype = ct.c_int
        L.oracle_term_test.argtypes = [vp, d, ct.c_int, d]
        L.oracle_term_test.restype = None
        L.oracle_canonical.argtypes = [vp, ct.c_int, vp]
        L.oracle_canonical.restype = None
        L.oracle_best.argtypes = [vp, vp, ct.c_int, ct.c_int, vp, vp, vp]
        L.oracle_best.restype = None
        L.oracle_brute_force.argtypes = [vp, ct.c_int, d, vp, vp, vp]
        L.oracle_brute_force.restype = lng
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ct.c_void_p)


def _c64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _ci32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def status_zero():
    return np.zeros(8, dtype=np.int32)


def correlate(R, status=None):
    """Pearson correlation of the demeaned rows of R (N x T), Eq. 7."""
    R = _c64(R)
    N, T = R.shape
    C = np.empty((N, N), dtype=np.float64)
    st = status if status is not None else status_zero()
    rc = lib().oracle_correlate(_p(R), N, T, T, _p(C), _p(st))
    if rc != 0:
        raise ValueError(f"oracle_correlate rc={rc}")
    return C


def fitness(C, pop, want_ns=False, want_cs=False, want_mag=False, status=None):
    """L_c (Eq. 8) of every row of pop (P x N). Returns fit, plus n_s, c_s, mag if asked."""
    C = _c64(C)
    pop = _ci32(np.atleast_2d(pop))
    P, N = pop.shape
    assert C.shape == (N, N)
    fit = np.empty(P, dtype=np.float64)
    ns = np.empty((P, N), dtype=np.int32) if want_ns else None
    cs = np.empty((P, N), dtype=np.float64) if want_cs else None
    mag = np.empty(P, dtype=np.float64) if want_mag else None
    st = status if status is not None else status_zero()
    lib().oracle_fitness(_p(C), N, _p(pop), P, _p(fit),
                         _p(ns) if ns is not None else None,
                         _p(cs) if cs is not None else None,
                         _p(mag) if mag is not None else None, _p(st))
    out = [fit]
    if want_ns:
        out.append(ns)
    if want_cs:
        out.append(cs)
    if want_mag:
        out.append(mag)
    return out[0] if len(out) == 1 else tuple(out)


def split_bf16(C):
    """(hi, lo) uint16 bfloat16 bit patterns with hi = bf16(C), lo = bf16(C - hi)."""
    C = _c64(C)
    hi = np.empty(C.shape, dtype=np.uint16)
    lo = np.empty(C.shape, dtype=np.uint16)
    lib().oracle_split_bf16(_p(C), C.size, _p(hi), _p(lo))
    return hi, lo


def bf16_to_f64(bits):
    """Decode bfloat16 bit patterns to float64 (exact)."""
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def philox(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def init_pop(N, P, seed=0, inst=0, gen0=0):
    pop = np.empty((P, N), dtype=np.int32)
    lib().oracle_init_pop(N, P, seed, inst, gen0, _p(pop))
    return pop


def rank(f):
    f = _c64(f)
    order = np.empty(f.shape[0], dtype=np.int32)
    lib().oracle_rank(_p(f), f.shape[0], _p(order))
    return order


def mut_thr(N):
    """Per-gene mutation threshold for probability 1/N: floor(2^32 / N)."""
    return (2**32) // N if N > 1 else 2**32 - 1


def breed(pop, f, E=2, p_cross_thr=P_CROSS_DEFAULT, p_mut_thr=None, seed=0, inst=0, gen=0, selection=0):
    """One replacement step; selection 0 = tournaments of two, 1 = stochastic universal sampling."""
    pop = _ci32(pop)
    f = _c64(f)
    P, N = pop.shape
    if p_mut_thr is None:
        p_mut_thr = mut_thr(N)
    out = np.empty_like(pop)
    lib().oracle_breed_sel(_p(pop), _p(f), N, P, E, selection, p_cross_thr, p_mut_thr, seed, inst, gen,
                           _p(out))
    return out


def sus_parents(f, E=2, seed=0, inst=0, gen=0):
    """Parents (2(P-E),) chosen by stochastic universal sampling after rank scaling."""
    f = _c64(f)
    P = f.shape[0]
    out = np.empty(max(0, 2 * (P - E)), dtype=np.int32)
    lib().oracle_sus_parents(_p(f), P, E, seed, inst, gen, _p(out))
    return out


def shuffle_index(x, n, seed=0, inst=0, gen=0):
    """Image of x under the Philox-keyed permutation of [0, n) used to pair SUS parents."""
    return int(lib().oracle_shuffle_index(x, n, seed, inst, gen))


def stats(f):
    f = _c64(f)
    out = np.empty(4, dtype=np.float64)
    lib().oracle_stats(_p(f), f.shape[0], _p(out))
    return out


def evolve(C, P, G, E=2, p_cross_thr=P_CROSS_DEFAULT, p_mut_thr=None, seed=0, inst=0, gen0=0,
           pop=None, status=None):
    """G generations (Algorithm 1) then a final fitness. Returns (pop, fit, stats[(G+1) x 4])."""
    C = _c64(C)
    N = C.shape[0]
    if p_mut_thr is None:
        p_mut_thr = mut_thr(N)
    init = pop is None
    pop = np.empty((P, N), dtype=np.int32) if init else _ci32(pop).copy()
    fit = np.empty(P, dtype=np.float64)
    st = np.empty((G + 1, 4), dtype=np.float64)
    status = status if status is not None else status_zero()
    rc = lib().oracle_evolve(_p(C), N, P, E, p_cross_thr, p_mut_thr, seed, inst, gen0, G, int(init),
                             _p(pop), _p(fit), _p(st), _p(status))
    if rc != 0:
        raise ValueError(f"oracle_evolve rc={rc}")
    return pop, fit, st


def evolve_term(C, P, G, stall_gens, tol, E=2, p_cross_thr=P_CROSS_DEFAULT, p_mut_thr=None, seed=0,
                inst=0, gen0=0, pop=None, state=None, status=None, selection=0):
    """Algorithm 1 with its termination test (Table 3: tolerance, stall generations).

    Returns (pop, fit, stats[(G+1) x 4], state) with state = [ref, stall, stopped, gens];
    statistics rows after a stop stay NaN. pop=None initialises the population (and
    the state); otherwise pass the state of the previous call to continue it."""
    C = _c64(C)
    N = C.shape[0]
    if p_mut_thr is None:
        p_mut_thr = mut_thr(N)
    init = pop is None
    pop = np.empty((P, N), dtype=np.int32) if init else _ci32(pop).copy()
    st8 = np.array([-np.inf, 0, 0, 0], dtype=np.float64) if state is None else _c64(state).copy()
    fit = np.empty(P, dtype=np.float64)
    st = np.full((G + 1, 4), np.nan, dtype=np.float64)
    status = status if status is not None else status_zero()
    rc = lib().oracle_evolve_term(_p(C), N, P, E, selection, p_cross_thr, p_mut_thr, seed, inst, gen0, G,
                                  int(init), stall_gens, float(tol), _p(pop), _p(fit), _p(st), _p(status),
                                  _p(st8))
    if rc != 0:
        raise ValueError(f"oracle_evolve_term rc={rc}")
    return pop, fit, st, st8


def term_test(state, b, stall_gens, tol):
    """The termination test of one evaluated generation with best fitness b; returns the new
    state [ref, stall, stopped, gens] (the input is not modified)."""
    st = _c64(state).copy()
    lib().oracle_term_test(_p(st), float(b), int(stall_gens), float(tol))
    return st


def ewma(R, lam=0.98, S=None, market=True, status=None):
    """Online EWMA correlation (Section 4.2.5): returns (C, S). S=None starts from a zero state;
    otherwise the recursion continues from the given state (not modified)."""
    R = _c64(R)
    N, T = R.shape
    reset = S is None
    S = np.zeros((N, N), dtype=np.float64) if reset else _c64(S).copy()
    C = np.empty((N, N), dtype=np.float64)
    status = status if status is not None else status_zero()
    lib().oracle_ewma(_p(R), N, T, T, float(lam), int(reset), int(market), _p(S), _p(C), _p(status))
    return C, S


def canonical(lab):
    lab = _ci32(lab)
    out = np.empty_like(lab)
    lib().oracle_canonical(_p(lab), lab.shape[0], _p(out))
    return out


def best(f, pop):
    f = _c64(f)
    pop = _ci32(pop)
    P, N = pop.shape
    lab = np.empty(N, dtype=np.int32)
    bf = np.zeros(1, dtype=np.float64)
    idx = np.zeros(1, dtype=np.int32)
    lib().oracle_best(_p(f), _p(pop), P, N, _p(lab), _p(bf), _p(idx))
    return lab, float(bf[0]), int(idx[0])


def brute_force(C, tie_tol=1e-12):
    """Maximum of L_c over every set partition. Returns (best_f, best_labels, n_best, n_visited)."""
    C = _c64(C)
    N = C.shape[0]
    lab = np.empty(N, dtype=np.int32)
    bf = np.zeros(1, dtype=np.float64)
    nb = np.zeros(1, dtype=np.int64)
    cnt = lib().oracle_brute_force(_p(C), N, tie_tol, _p(bf), _p(lab), _p(nb))
    if cnt < 0:
        raise ValueError("brute force supports 1 <= N <= 14")
    return float(bf[0]), lab, int(nb[0]), int(cnt)
