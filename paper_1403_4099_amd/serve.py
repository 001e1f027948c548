"""Continuous-batching request loop for streams of correlation windows.

A request is one correlation window (returns R, N x T) of a *universe* (a fixed
set of stocks). Each universe keeps its GA population resident on the GPU:
a new window of the same universe warm-starts from the population the
previous one ended with (Algorithm 1 continued on fresh data), so intraday
re-clustering does not restart from random labelings.

Scheduling (host side; every computation is a libpga kernel):
  * arrivals are admitted FIFO when the universe has no request in flight
    and the HBM footprint of the new request fits the budget (otherwise they
    wait; a request whose footprint alone exceeds the budget is rejected).
    The budget counts the in-flight requests' transient buffers and every
    resident population (P x N int32 per universe, kept between windows);
    when an arrival does not fit, resident populations of idle universes are
    evicted, least recently used first, and such a universe's next window
    starts from a fresh initial population;
  * admitted requests get their correlation matrix (pga_correlate), then all
    requests in flight advance together by `chunk` generations in ONE
    pga_evolve call over the ragged set of instances (different N);
  * a request that has done its generations is retired with pga_best
    (canonical labels) and its latency (arrival -> result) is recorded;
    with the GA's termination test on (stall generations and tolerance,
    Table 3) a request whose GA has stopped retires at the next chunk
    boundary instead; new arrivals join at the next chunk boundary
    (continuous batching).
Random draws are keyed by (universe id, absolute generation), and evolving
g1 then g2 generations equals g1 + g2 at once, so every result is bit-for-bit
the same whether a request ran alone or in a mix.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Request:
    rid: int
    universe: int
    arrival: float          # seconds from the start of the stream
    R: object               # device tensor N x T (float64)
    N: int
    T: int


@dataclass
class Result:
    rid: int
    universe: int
    arrival: float
    admitted: float
    done: float
    labels: np.ndarray
    fitness: float
    gen_end: int

    @property
    def latency(self) -> float:
        return self.done - self.arrival


def resident_bytes(N: int, P: int) -> int:
    """HBM bytes of a universe's resident population (P x N int32), kept between windows."""
    return 4 * P * N


def footprint_bytes(N: int, P: int, split_ld: int, form: str) -> int:
    """HBM bytes one in-flight request holds besides its universe's resident population: C,
    BF16 split, the population's ping-pong partner, fitness, stats, and its share of the evolve
    workspace (pair sums P x N FP64, elites, descriptor, and for the BF16x2 form the scaled
    split copies)."""
    b = 8 * N * N + 8 * P + 8 * N * P + 4096
    b += 4 * P * N                          # ping-pong partner of the population
    if form == "bf16x2":
        b += 2 * 2 * split_ld * split_ld    # hi, lo
        b += 2 * 2 * split_ld * split_ld    # their scaled workspace copies
    return b


@dataclass
class _Flight:
    req: Request
    inst: object
    C: object
    hi: object
    lo: object
    remaining: int
    admitted: float
    bytes: int


class Scheduler:
    """Admission, chunking and retirement. `engine` does the device work:
       engine.start(req, gen0, warm_pop) -> (inst, C, hi, lo)
       engine.advance(list_of_inst, generations)
       engine.progress(list_of_inst) -> [(stopped, generations bred so far)] (one sync)
       engine.finish(inst) -> (labels, fitness)
       engine.resident(universe) -> population tensor or None
       engine.keep(universe, inst) -> keeps the final population resident
       engine.evict(universe) -> drops a resident population
    """

    def __init__(self, engine, P: int = 1024, generations: int = 100, chunk: int = 10,
                 hbm_budget: int = 8 << 30, form: str = "fp64", split_ld=lambda n: (n + 31) // 32 * 32,
                 clock=time.perf_counter):
        assert generations % chunk == 0
        self.engine = engine
        self.P, self.G, self.chunk = P, generations, chunk
        self.budget = hbm_budget
        self.form = form
        self.split_ld = split_ld
        self.clock = clock
        self.pending: collections.deque[Request] = collections.deque()
        self.flights: list[_Flight] = []
        self.busy: set[int] = set()
        self.gen_of: dict[int, int] = collections.defaultdict(int)
        self.used = 0                       # in-flight transient bytes + resident populations
        self.resident: collections.OrderedDict[int, int] = collections.OrderedDict()   # universe -> bytes (LRU)
        self.evictions = 0
        self.results: list[Result] = []
        self.rejected: list[Request] = []
        self.t0 = None
        self.max_inflight = 0
        self.chunks_run = 0

    def now(self) -> float:
        return self.clock() - self.t0

    def _make_room(self, need: int, keep: int) -> bool:
        """Evict idle residents (least recently used first, never `keep`) until `need` more
        bytes fit; True if they do."""
        for u in list(self.resident):
            if self.used + need <= self.budget:
                break
            if u == keep or u in self.busy:
                continue
            self.used -= self.resident.pop(u)
            self.engine.evict(u)
            self.evictions += 1
        return self.used + need <= self.budget

    def _admit(self):
        kept = collections.deque()
        while self.pending:
            r = self.pending.popleft()
            need = footprint_bytes(r.N, self.P, self.split_ld(r.N), self.form)
            res = 0 if r.universe in self.resident else resident_bytes(r.N, self.P)
            if need + resident_bytes(r.N, self.P) > self.budget:
                self.rejected.append(r)
                continue
            if r.universe in self.busy or not self._make_room(need + res, r.universe):
                kept.append(r)
                continue
            gen0 = self.gen_of[r.universe]
            inst, C, hi, lo = self.engine.start(r, gen0, self.engine.resident(r.universe))
            self.flights.append(_Flight(r, inst, C, hi, lo, self.G, self.now(), need))
            self.busy.add(r.universe)
            self.used += need + res
            self.resident[r.universe] = resident_bytes(r.N, self.P)
            self.resident.move_to_end(r.universe)
        self.pending = kept
        self.max_inflight = max(self.max_inflight, len(self.flights))

    def _advance(self):
        insts = [f.inst for f in self.flights]
        self.engine.advance(insts, self.chunk)
        self.chunks_run += 1
        prog = self.engine.progress(insts)
        still = []
        for f, (stopped, bred) in zip(self.flights, prog):
            f.remaining -= self.chunk
            if f.remaining > 0 and not stopped:
                still.append(f)
                continue
            labels, fit = self.engine.finish(f.inst)
            u = f.req.universe
            self.gen_of[u] += bred if bred is not None else self.G
            self.engine.keep(u, f.inst)
            self.busy.discard(u)
            self.used -= f.bytes
            self.results.append(Result(f.req.rid, u, f.req.arrival, f.admitted, self.now(), labels, fit,
                                       self.gen_of[u]))
        self.flights = still

    def run(self, requests: list[Request]) -> list[Result]:
        """Serve `requests` (sorted by arrival time, seconds from start) in real time."""
        arrivals = sorted(requests, key=lambda r: r.arrival)
        i = 0
        self.t0 = self.clock()
        while i < len(arrivals) or self.pending or self.flights:
            now = self.now()
            while i < len(arrivals) and arrivals[i].arrival <= now:
                self.pending.append(arrivals[i])
                i += 1
            self._admit()
            if self.flights:
                self._advance()
            elif i < len(arrivals):
                wait = arrivals[i].arrival - self.now()
                if wait > 0:
                    time.sleep(min(wait, 0.002))
            elif self.pending:
                # nothing in flight but requests wait: only possible if the budget never fits
                self.rejected.extend(self.pending)
                self.pending.clear()
        return self.results

    def summary(self) -> dict:
        lat = np.array([r.latency for r in self.results]) if self.results else np.zeros(1)
        span = max((r.done for r in self.results), default=0.0)
        return {
            "requests": len(self.results),
            "rejected": len(self.rejected),
            "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "mean_ms": float(lat.mean() * 1e3),
            "requests_per_s": len(self.results) / span if span > 0 else 0.0,
            "max_in_flight": self.max_inflight,
            "chunks": self.chunks_run,
            "evictions": self.evictions,
        }


class GpuEngine:
    """libpga-backed engine: correlation, warm-started ragged evolve, best."""

    def __init__(self, P: int = 1024, form: str = "fp64", elites: int = 2, seed: int = 0,
                 eager: bool = False, stall_gens: int = 0, tol: float = 1e-5):
        import torch

        from . import pga
        self.pga = pga
        self.torch = torch
        self.P, self.form, self.E, self.seed = P, form, elites, seed
        self.eager = eager
        self.stall_gens, self.tol = stall_gens, tol
        self.ctx = pga.Context()
        # one workspace for every mix of requests (grown only if a mix needs more), so the
        # graphs captured for the chunk launches stay valid from one mix to the next
        self.ctx.ws = torch.empty(128 << 20, dtype=torch.uint8, device="cuda")
        self.pops: dict[int, object] = {}
        self.status = pga.new_status()

    def resident(self, universe):
        return self.pops.get(universe)

    def start(self, req: Request, gen0: int, warm_pop):
        pga, torch = self.pga, self.torch
        split = self.form == "bf16x2"
        out = pga.correlate(req.R, split=split, status=self.status)
        C, hi, lo = out if split else (out, None, None)
        init = warm_pop is None
        pop = torch.empty((self.P, req.N), dtype=torch.int32, device=C.device) if init else warm_pop
        inst = pga.make_instance(C, self.P, hi=hi, lo=lo, pop=pop, elites=self.E, seed=self.seed,
                                 instance_id=req.universe, gen0=gen0, stall_gens=self.stall_gens,
                                 tol=self.tol)
        if init:
            self.ctx.evolve([inst], 0, form=self.form, init=True, eager=True, status=self.status)
        return inst, C, hi, lo

    def advance(self, insts, generations):
        self.ctx.evolve(insts, generations, form=self.form, eager=self.eager, status=self.status)
        for inst in insts:
            inst.gen0 += generations

    def progress(self, insts):
        """[(stopped, generations bred since start)] of each instance; None counts without the test."""
        if self.stall_gens <= 0:
            return [(False, None)] * len(insts)
        raw = self.torch.stack([i.term for i in insts]).cpu().numpy()
        out = []
        for row in raw:
            ts = self.pga.TermState.from_buffer_copy(row.tobytes())
            out.append((bool(ts.stopped), int(ts.gens)))
        return out

    def finish(self, inst):
        labels, f, _ = self.pga.best(inst.fitness, inst.pop)
        return labels, f

    def keep(self, universe, inst):
        self.pops[universe] = inst.pop

    def evict(self, universe):
        self.pops.pop(universe, None)
