"""Python binding of libpga (ctypes). Argument marshalling only.

Every step of the path runs in the HIP kernels of libpga.so; this module
passes device pointers of torch tensors and the current HIP stream through
the C ABI declared in include/pga.h, and allocates device buffers with
torch. There is no CPU fallback: if libpga.so is missing or no GPU is
present, calls raise.
"""
from __future__ import annotations

import ctypes as ct
import os
from dataclasses import dataclass

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpga.so")

PGA_OK = 0
FORM_FP64 = 0
FORM_BF16X2 = 1
FORMS = {"fp64": FORM_FP64, "bf16x2": FORM_BF16X2}
SELECTIONS = {"tournament": 0, "sus": 1}
STATUS_WORDS = 8
ST_LABEL, ST_DOMAIN, ST_ZEROVAR, ST_NONFINITE = 0, 1, 2, 3
N_MAX = 4096
E_MAX = 64
EVOLVE_INIT = 1
EVOLVE_EAGER = 2
P_CROSS_DEFAULT = int(0.9 * 2**32)
KERNELS = {"pairsum_fp64": 0, "pairsum_mfma": 1, "finish": 2, "rank": 3, "breed": 4,
           "correlate": 5, "split": 6, "init": 7, "sus": 8, "ewma": 9, "cluster_pairs": 10, "nsmask": 11}
EWMA_RESET, EWMA_MARKET = 1, 2

SYMBOLS = [
    "pga_ctx_create", "pga_ctx_destroy", "pga_ctx_graphs", "pga_strerror", "pga_last_hip_error",
    "pga_correlate_ws_bytes", "pga_correlate", "pga_split_ld", "pga_split",
    "pga_fitness_ws_bytes", "pga_fitness", "pga_evolve_ws_bytes", "pga_evolve",
    "pga_best_ws_bytes", "pga_best", "pga_timing_enable", "pga_timing_reset", "pga_timing_read",
    "pga_variant_count", "pga_variant_info", "pga_tune_ws_bytes", "pga_tune", "pga_tune_set",
    "pga_tune_get", "pga_tune_save", "pga_tune_load", "pga_ewma_ws_bytes", "pga_ewma", "pga_peak_mfma_bf16", "pga_route_set",
    "pga_route_get", "pga_fitness_noalloc", "pga_fitness_noalloc_max_bytes", "pga_peak_fp64", "pga_pipe_mix",
]


class PgaError(RuntimeError):
    pass


class Params(ct.Structure):
    _fields_ = [("elites", ct.c_int32), ("tournament", ct.c_int32), ("p_cross_thr", ct.c_uint32),
                ("p_mut_thr", ct.c_uint32), ("seed", ct.c_uint64), ("instance_id", ct.c_uint32),
                ("gen0", ct.c_uint32), ("stall_gens", ct.c_int32), ("selection", ct.c_int32),
                ("tol", ct.c_double)]


class TermState(ct.Structure):
    """pga_term_state (device memory; read back with Instance.term_state())."""
    _fields_ = [("ref", ct.c_double), ("stall", ct.c_int32), ("stopped", ct.c_int32),
                ("gens", ct.c_int32), ("call_gens", ct.c_int32)]


class InstanceC(ct.Structure):
    _fields_ = [("N", ct.c_int32), ("P", ct.c_int32), ("C", ct.c_void_p), ("C_hi", ct.c_void_p),
                ("C_lo", ct.c_void_p), ("pop", ct.c_void_p), ("pop_tmp", ct.c_void_p),
                ("fitness", ct.c_void_p), ("stats", ct.c_void_p), ("term", ct.c_void_p), ("prm", Params)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libpga.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise PgaError(f"{path} not found: build it with paper_1403_4099_amd/build.py")
    L = ct.CDLL(path)
    vp, i32, i64, sz = ct.c_void_p, ct.c_int32, ct.c_int64, ct.c_size_t
    sig = {
        "pga_ctx_create": ([ct.POINTER(vp)], ct.c_int),
        "pga_ctx_destroy": ([vp], ct.c_int),
        "pga_ctx_graphs": ([vp], ct.c_int),
        "pga_strerror": ([ct.c_int], ct.c_char_p),
        "pga_last_hip_error": ([], ct.c_int),
        "pga_correlate_ws_bytes": ([i32], sz),
        "pga_correlate": ([vp, i32, i32, i64, vp, vp, vp, vp, vp, sz, vp], ct.c_int),
        "pga_split_ld": ([i32], i32),
        "pga_split": ([vp, i32, vp, vp, vp], ct.c_int),
        "pga_fitness_ws_bytes": ([i32, i32, i32], sz),
        "pga_fitness": ([vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, sz, vp], ct.c_int),
        "pga_evolve_ws_bytes": ([ct.POINTER(InstanceC), i32, i32], sz),
        "pga_evolve": ([vp, ct.POINTER(InstanceC), i32, i32, i32, i32, vp, sz, vp, vp], ct.c_int),
        "pga_best_ws_bytes": ([i32], sz),
        "pga_best": ([vp, vp, i32, i32, vp, vp, vp, vp, sz, vp], ct.c_int),
        "pga_timing_enable": ([ct.c_int], ct.c_int),
        "pga_timing_reset": ([], ct.c_int),
        "pga_timing_read": ([ct.c_int, ct.POINTER(ct.c_double), ct.POINTER(ct.c_int64)], ct.c_int),
        "pga_variant_count": ([i32], ct.c_int),
        "pga_variant_info": ([i32, i32, ct.POINTER(i32), ct.POINTER(i32), ct.POINTER(i32)], ct.c_int),
        "pga_tune_ws_bytes": ([i32, i32, i32], sz),
        "pga_tune": ([vp, vp, vp, i32, vp, i32, i32, i32, vp, sz, ct.POINTER(i32), ct.POINTER(ct.c_float), vp],
                     ct.c_int),
        "pga_tune_set": ([i32, i32, i32, i32], ct.c_int),
        "pga_tune_get": ([i32, i32, i32], ct.c_int),
        "pga_tune_save": ([ct.c_char_p], ct.c_int),
        "pga_tune_load": ([ct.c_char_p], ct.c_int),
        "pga_ewma_ws_bytes": ([i32, i32], sz),
        "pga_ewma": ([vp, i32, i32, i32, ct.c_double, i32, vp, vp, vp, vp, vp, vp, sz, vp], ct.c_int),
        "pga_peak_mfma_bf16": ([vp, i32, i32, ct.POINTER(ct.c_double), vp], ct.c_int),
        "pga_peak_fp64": ([vp, i32, i32, ct.POINTER(ct.c_double), vp], ct.c_int),
        "pga_pipe_mix": ([vp, i32, i32, i32, vp], ct.c_int),
        "pga_route_set": ([ct.c_double], ct.c_int),
        "pga_route_get": ([], ct.c_double),
        "pga_fitness_noalloc": ([vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp], ct.c_int),
        "pga_fitness_noalloc_max_bytes": ([], sz),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def _check(rc: int, what: str):
    if rc != PGA_OK:
        L = load()
        msg = L.pga_strerror(rc).decode()
        hip = L.pga_last_hip_error() if rc == -3 else None
        raise PgaError(f"{what}: {msg} (rc={rc}{', hip=' + str(hip) if hip is not None else ''})")


def _ptr(t):
    return None if t is None else ct.c_void_p(t.data_ptr())


def _stream(device=None):
    return ct.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev():
    if not torch.cuda.is_available():
        raise PgaError("no GPU visible: libpga needs an MI355X (gfx950)")
    return torch.device("cuda", torch.cuda.current_device())


def _workspace(nbytes: int, device) -> torch.Tensor:
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def new_status(device=None) -> torch.Tensor:
    return torch.zeros(STATUS_WORDS, dtype=torch.int32, device=device or _dev())


def split_ld(N: int) -> int:
    return int(load().pga_split_ld(N))


def mut_thr(N: int) -> int:
    return (2**32) // N if N > 1 else 2**32 - 1


# ---------------------------------------------------------------- correlation and split
def correlate(R: torch.Tensor, split: bool = False, status: torch.Tensor | None = None):
    """Pearson correlation of the rows of R (N x T, float64, on the GPU). Returns C or (C, hi, lo)."""
    L = load()
    dev = _dev()
    assert R.is_cuda and R.dtype == torch.float64 and R.dim() == 2 and R.stride(1) == 1
    N, T = R.shape
    C = torch.empty((N, N), dtype=torch.float64, device=dev)
    hi = lo = None
    if split:
        ld = split_ld(N)
        hi = torch.empty((ld, ld), dtype=torch.int16, device=dev)
        lo = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    ws = _workspace(L.pga_correlate_ws_bytes(N), dev)
    rc = L.pga_correlate(_ptr(R), N, T, R.stride(0), _ptr(C), _ptr(hi), _ptr(lo), _ptr(status),
                         _ptr(ws), ws.numel(), _stream())
    _check(rc, "pga_correlate")
    return (C, hi, lo) if split else C


def split(C: torch.Tensor):
    """BF16 hi + lo split of C (N x N float64) into split_ld(N)^2 int16 bit-pattern arrays."""
    L = load()
    dev = _dev()
    N = C.shape[0]
    ld = split_ld(N)
    hi = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    lo = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    _check(L.pga_split(_ptr(C), N, _ptr(hi), _ptr(lo), _stream()), "pga_split")
    return hi, lo


# ---------------------------------------------------------------- fitness
def fitness(C: torch.Tensor, labels: torch.Tensor, form: str = "fp64", hi=None, lo=None,
            want_ns: bool = False, want_cs: bool = False, status: torch.Tensor | None = None,
            out: torch.Tensor | None = None, ws: torch.Tensor | None = None):
    """L_c of every row of labels (P x N int32). Returns fitness (P,) [, n_s (P x N), c_s (P x N)]."""
    L = load()
    dev = _dev()
    P, N = labels.shape
    assert labels.dtype == torch.int32 and labels.is_contiguous()
    f = out if out is not None else torch.empty(P, dtype=torch.float64, device=dev)
    ns = torch.empty((P, N), dtype=torch.int32, device=dev) if want_ns else None
    cs = torch.empty((P, N), dtype=torch.float64, device=dev) if want_cs else None
    need = L.pga_fitness_ws_bytes(N, P, FORMS[form])
    if ws is None or ws.numel() < need:
        ws = _workspace(need, dev)
    rc = L.pga_fitness(_ptr(C), _ptr(hi), _ptr(lo), N, _ptr(labels), P, FORMS[form], _ptr(f),
                       _ptr(ns), _ptr(cs), _ptr(status), _ptr(ws), ws.numel(), _stream())
    _check(rc, "pga_fitness")
    res = [f]
    if want_ns:
        res.append(ns)
    if want_cs:
        res.append(cs)
    return res[0] if len(res) == 1 else tuple(res)


def fitness_noalloc(C: torch.Tensor, labels: torch.Tensor, form: str = "fp64", hi=None, lo=None,
                    want_ns: bool = False, want_cs: bool = False, status: torch.Tensor | None = None,
                    out: torch.Tensor | None = None):
    """As fitness(), through pga_fitness_noalloc (scratch in the library's static device array;
    the library allocates nothing). Output tensors are allocated here unless passed in."""
    L = load()
    dev = _dev()
    P, N = labels.shape
    assert labels.dtype == torch.int32 and labels.is_contiguous()
    f = out if out is not None else torch.empty(P, dtype=torch.float64, device=dev)
    ns = torch.empty((P, N), dtype=torch.int32, device=dev) if want_ns else None
    cs = torch.empty((P, N), dtype=torch.float64, device=dev) if want_cs else None
    rc = L.pga_fitness_noalloc(_ptr(C), _ptr(hi), _ptr(lo), N, _ptr(labels), P, FORMS[form], _ptr(f),
                               _ptr(ns), _ptr(cs), _ptr(status), _stream())
    _check(rc, "pga_fitness_noalloc")
    res = [f]
    if want_ns:
        res.append(ns)
    if want_cs:
        res.append(cs)
    return res[0] if len(res) == 1 else tuple(res)


def noalloc_max_bytes() -> int:
    return int(load().pga_fitness_noalloc_max_bytes())


def fitness_ws_bytes(N: int, P: int, form: str = "fp64") -> int:
    return int(load().pga_fitness_ws_bytes(N, P, FORMS[form]))


# ---------------------------------------------------------------- EWMA correlation
def ewma(R: torch.Tensor, S: torch.Tensor, lam: float = 0.98, reset: bool = False, market: bool = True,
         split: bool = False, status: torch.Tensor | None = None):
    """Online EWMA correlation (pga_ewma). Updates S (N x N) in place; returns C [, hi, lo]."""
    L = load()
    dev = _dev()
    N, T = R.shape
    assert R.dtype == torch.float64 and R.stride(1) == 1 and S.shape == (N, N) and S.is_contiguous()
    C = torch.empty((N, N), dtype=torch.float64, device=dev)
    hi = lo = None
    if split:
        ld = split_ld(N)
        hi = torch.empty((ld, ld), dtype=torch.int16, device=dev)
        lo = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    ws = _workspace(L.pga_ewma_ws_bytes(N, T), dev)
    flags = (EWMA_RESET if reset else 0) | (EWMA_MARKET if market else 0)
    rc = L.pga_ewma(_ptr(R), N, T, R.stride(0), float(lam), flags, _ptr(S), _ptr(C), _ptr(hi), _ptr(lo),
                    _ptr(status), _ptr(ws), ws.numel(), _stream())
    _check(rc, "pga_ewma")
    return (C, hi, lo) if split else C


# ---------------------------------------------------------------- autotuning
def variants(form: str = "fp64"):
    """[(individuals per group, xcd order, kind)] of the pair-sum kernel variants of a form
    (kind, MFMA form only: 0 per-stock columns, one-hot built in registers; 1 compacted columns;
    2 per-stock columns, one-hot read from an LDS table)."""
    L = load()
    n = L.pga_variant_count(FORMS[form])
    out = []
    for v in range(n):
        ipg, xcd, kind = ct.c_int32(), ct.c_int32(), ct.c_int32()
        _check(L.pga_variant_info(FORMS[form], v, ct.byref(ipg), ct.byref(xcd), ct.byref(kind)),
               "pga_variant_info")
        out.append((ipg.value, xcd.value, kind.value))
    return out


def tune(C: torch.Tensor, labels: torch.Tensor, form: str = "fp64", hi=None, lo=None, reps: int = 5):
    """SYNC. Time every variant on labels, record the fastest; returns (variant, [ms per variant])."""
    L = load()
    dev = _dev()
    P, N = labels.shape
    need = L.pga_tune_ws_bytes(N, P, FORMS[form])
    if need == 0:
        raise PgaError("pga_tune_ws_bytes: invalid shape or form")
    ws = _workspace(need, dev)
    n = L.pga_variant_count(FORMS[form])
    ms = (ct.c_float * n)()
    v = ct.c_int32(-1)
    rc = L.pga_tune(_ptr(C), _ptr(hi), _ptr(lo), N, _ptr(labels), P, FORMS[form], reps, _ptr(ws),
                    ws.numel(), ct.byref(v), ms, _stream())
    _check(rc, "pga_tune")
    return v.value, [float(x) for x in ms]


def route_set(frac: float):
    """Cluster-pair route limit: individuals with at most frac * N (N - 1) / 2
    within-cluster pairs (and N <= 2048) skip the O(N^2) pair-sum; 0 = off."""
    _check(load().pga_route_set(float(frac)), "pga_route_set")


def route_get() -> float:
    return float(load().pga_route_get())


class route:
    """Context manager: run a block with another route limit, then restore it."""

    def __init__(self, frac: float):
        self.frac = frac

    def __enter__(self):
        self.prev = route_get()
        route_set(self.frac)
        return self

    def __exit__(self, *exc):
        route_set(self.prev)
        return False


def tune_set(form: str, N: int, P: int, variant: int):
    _check(load().pga_tune_set(FORMS[form], N, P, variant), "pga_tune_set")


def tune_save(path: str) -> int:
    """Write the tuning table to a text file; returns the number of entries."""
    n = load().pga_tune_save(os.fsencode(path))
    if n < 0:
        _check(n, "pga_tune_save")
    return n


def tune_load(path: str) -> int:
    """Add the entries of a tuning-table file; returns their number."""
    n = load().pga_tune_load(os.fsencode(path))
    if n < 0:
        _check(n, "pga_tune_load")
    return n


def tune_get(form: str, N: int, P: int) -> int:
    v = load().pga_tune_get(FORMS[form], N, P)
    if v < 0:
        _check(v, "pga_tune_get")
    return v


# ---------------------------------------------------------------- evolution
@dataclass
class Instance:
    """One GA instance: device buffers plus parameters (Algorithm 1 state)."""
    C: torch.Tensor
    pop: torch.Tensor
    pop_tmp: torch.Tensor
    fitness: torch.Tensor
    hi: torch.Tensor | None = None
    lo: torch.Tensor | None = None
    stats: torch.Tensor | None = None
    elites: int = 2
    p_cross_thr: int = P_CROSS_DEFAULT
    p_mut_thr: int | None = None
    seed: int = 0
    instance_id: int = 0
    gen0: int = 0
    stall_gens: int = 0
    tol: float = 1e-5
    selection: str = "tournament"      # or "sus"
    term: torch.Tensor | None = None   # pga_term_state bytes (uint8, device)

    @property
    def N(self) -> int:
        return self.pop.shape[1]

    @property
    def P(self) -> int:
        return self.pop.shape[0]

    def to_c(self) -> InstanceC:
        pm = self.p_mut_thr if self.p_mut_thr is not None else mut_thr(self.N)
        prm = Params(self.elites, 2, self.p_cross_thr, pm, self.seed, self.instance_id, self.gen0,
                     self.stall_gens, SELECTIONS[self.selection], self.tol)
        return InstanceC(self.N, self.P, self.C.data_ptr(),
                         self.hi.data_ptr() if self.hi is not None else None,
                         self.lo.data_ptr() if self.lo is not None else None,
                         self.pop.data_ptr(), self.pop_tmp.data_ptr(), self.fitness.data_ptr(),
                         self.stats.data_ptr() if self.stats is not None else None,
                         self.term.data_ptr() if self.term is not None else None, prm)

    def term_state(self) -> dict:
        """SYNC. The termination state {ref, stall, stopped, gens, call_gens}."""
        if self.term is None:
            raise PgaError("instance has no termination state")
        raw = bytes(self.term.cpu().numpy().tobytes())
        ts = TermState.from_buffer_copy(raw[: ct.sizeof(TermState)])
        return {k: getattr(ts, k) for k, _ in TermState._fields_}


def make_instance(C, P, hi=None, lo=None, pop=None, stats_rows=0, **kw) -> Instance:
    dev = _dev()
    N = C.shape[0]
    if pop is None:
        pop = torch.empty((P, N), dtype=torch.int32, device=dev)
    st = torch.empty((stats_rows, 4), dtype=torch.float64, device=dev) if stats_rows else None
    fresh = bytes(TermState(float("-inf"), 0, 0, 0, 0))
    term = torch.frombuffer(bytearray(fresh), dtype=torch.uint8).to(dev)
    return Instance(C=C, hi=hi, lo=lo, pop=pop, pop_tmp=torch.empty_like(pop), term=term,
                    fitness=torch.empty(P, dtype=torch.float64, device=dev), stats=st, **kw)


class Context:
    """Owns a pga_ctx (captured HIP graphs, descriptor staging) and a reusable workspace."""

    def __init__(self):
        L = load()
        h = ct.c_void_p()
        _check(L.pga_ctx_create(ct.byref(h)), "pga_ctx_create")
        self.h = h
        self.ws = None

    def graphs(self) -> int:
        """Captured graphs held by the context."""
        n = load().pga_ctx_graphs(self.h)
        if n < 0:
            _check(n, "pga_ctx_graphs")
        return n

    def close(self):
        if self.h:
            load().pga_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def evolve(self, insts, generations: int, form: str = "fp64", init: bool = False,
               eager: bool = False, status: torch.Tensor | None = None):
        """Run `generations` generations on every instance (pga_evolve)."""
        L = load()
        dev = _dev()
        arr = (InstanceC * len(insts))(*[i.to_c() for i in insts])
        need = L.pga_evolve_ws_bytes(arr, len(insts), FORMS[form])
        if need == 0:
            raise PgaError("pga_evolve_ws_bytes: invalid instances")
        if self.ws is None or self.ws.numel() < need:
            self.ws = _workspace(need, dev)
        flags = (EVOLVE_INIT if init else 0) | (EVOLVE_EAGER if eager else 0)
        rc = L.pga_evolve(self.h, arr, len(insts), generations, FORMS[form], flags,
                          _ptr(self.ws), self.ws.numel(), _ptr(status), _stream())
        _check(rc, "pga_evolve")


# ---------------------------------------------------------------- result
def best(fitness_t: torch.Tensor, labels: torch.Tensor):
    """SYNC. (canonical labels as numpy int32, fitness, index) of the fittest labeling."""
    L = load()
    dev = _dev()
    P, N = labels.shape
    ws = _workspace(L.pga_best_ws_bytes(N), dev)
    out = np.empty(N, dtype=np.int32)
    f = ct.c_double()
    idx = ct.c_int32()
    rc = L.pga_best(_ptr(fitness_t), _ptr(labels), P, N, out.ctypes.data_as(ct.c_void_p),
                    ct.byref(f), ct.byref(idx), _ptr(ws), ws.numel(), _stream())
    _check(rc, "pga_best")
    return out, f.value, idx.value


# ---------------------------------------------------------------- measured ceiling
def peak_mfma_bf16(n_workgroups: int = 4096, iters: int = 1000, reps: int = 5) -> float:
    """Sustained bf16 MFMA throughput in TFLOP/s (best of `reps` timed launches of the library's
    register-operand MFMA loop on the current stream)."""
    out = torch.empty(4 * n_workgroups, dtype=torch.float32, device="cuda")
    flops = ct.c_double()
    L = load()
    _check(L.pga_peak_mfma_bf16(_ptr(out), n_workgroups, iters, ct.byref(flops), _stream()), "pga_peak_mfma_bf16")
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _check(L.pga_peak_mfma_bf16(_ptr(out), n_workgroups, iters, None, _stream()), "pga_peak_mfma_bf16")
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    if not bool(torch.isfinite(out).all()):
        raise PgaError("pga_peak_mfma_bf16: non-finite sink values")
    return flops.value / best / 1e12


def peak_fp64(n_workgroups: int = 4096, iters: int = 2000, reps: int = 5) -> float:
    """Sustained FP64 vector FMA throughput in TFLOP/s (best of `reps` timed launches of the
    library's register-operand FMA loop on the current stream)."""
    out = torch.empty(4 * n_workgroups, dtype=torch.float64, device="cuda")
    flops = ct.c_double()
    L = load()
    _check(L.pga_peak_fp64(_ptr(out), n_workgroups, iters, ct.byref(flops), _stream()), "pga_peak_fp64")
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        _check(L.pga_peak_fp64(_ptr(out), n_workgroups, iters, None, _stream()), "pga_peak_fp64")
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    if not bool(torch.isfinite(out).all()):
        raise PgaError("pga_peak_fp64: non-finite sink values")
    return flops.value / best / 1e12


PIPE_MIX_MODES = {"mfma": 1, "valu": 2, "mfma+valu": 3, "lds": 4, "mfma+lds": 5,
                  "mfma|valu": 11, "mfma|lds": 13}


def pipe_mix(n_workgroups: int = 2048, iters: int = 2000, reps: int = 3) -> dict:
    """Cycles per round per wave on one SIMD of each pipe-mix mode (pga_pipe_mix): the best of
    `reps` timed launches, converted at 2.4 GHz over the GPU's SIMDs (4 per compute unit).
    "a+b" runs both in every wave, "a|b" splits them over alternate waves."""
    out = torch.empty(4 * n_workgroups, dtype=torch.float32, device="cuda")
    L = load()
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    waves_per_simd = n_workgroups * 4 / simds
    res = {}
    for name, mode in PIPE_MIX_MODES.items():
        _check(L.pga_pipe_mix(_ptr(out), mode, n_workgroups, 10, _stream()), "pga_pipe_mix")
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            _check(L.pga_pipe_mix(_ptr(out), mode, n_workgroups, iters, _stream()), "pga_pipe_mix")
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        res[name] = best * 2.4e9 / (iters * waves_per_simd)
    if not bool(torch.isfinite(out).all()):
        raise PgaError("pga_pipe_mix: non-finite sink values")
    return res


# ---------------------------------------------------------------- timing
def timing_enable(on: bool = True):
    _check(load().pga_timing_enable(1 if on else 0), "pga_timing_enable")


def timing_reset():
    _check(load().pga_timing_reset(), "pga_timing_reset")


def timing_read(kernel: str):
    ms = ct.c_double()
    n = ct.c_int64()
    _check(load().pga_timing_read(KERNELS[kernel], ct.byref(ms), ct.byref(n)), "pga_timing_read")
    return ms.value, n.value
