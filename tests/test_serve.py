"""CPU tests of the continuous-batching scheduler's host logic with a fake engine
(admission by HBM budget with resident populations counted, eviction of idle residents,
one request per universe in flight, FIFO, retirement)."""
import numpy as np

from paper_1403_4099_amd.serve import Request, Scheduler, footprint_bytes, resident_bytes


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t


class FakeEngine:
    def __init__(self, clock, cost_per_gen=1e-4, stop_after=None):
        self.clock = clock
        self.cost = cost_per_gen
        self.pops = {}
        self.log = []
        self.stop_after = stop_after or {}     # rid -> generations after which the GA stops

    def resident(self, u):
        return self.pops.get(u)

    def start(self, req, gen0, warm):
        self.log.append(("start", req.rid, req.universe, gen0, warm is not None))
        return {"req": req, "gen": gen0, "bred": 0}, None, None, None

    def advance(self, insts, g):
        self.log.append(("advance", tuple(i["req"].rid for i in insts), g))
        self.clock.t += self.cost * g * len(insts)
        for i in insts:
            lim = self.stop_after.get(i["req"].rid)
            step = g if lim is None else max(0, min(g, lim - i["bred"]))
            i["gen"] += step
            i["bred"] += step

    def progress(self, insts):
        out = []
        for i in insts:
            lim = self.stop_after.get(i["req"].rid)
            out.append((lim is not None and i["bred"] >= lim, i["bred"] if self.stop_after else None))
        return out

    def finish(self, inst):
        return np.zeros(inst["req"].N, dtype=np.int32), float(inst["gen"])

    def keep(self, u, inst):
        self.pops[u] = inst["gen"]

    def evict(self, u):
        self.log.append(("evict", u))
        self.pops.pop(u, None)


def _reqs(spec):
    return [Request(i, u, t, None, N, 390) for i, (t, u, N) in enumerate(spec)]


def test_all_requests_complete_and_universes_do_not_overlap():
    clk = FakeClock()
    eng = FakeEngine(clk)
    s = Scheduler(eng, P=64, generations=20, chunk=5, hbm_budget=1 << 30, clock=clk)
    reqs = _reqs([(0.0, 0, 64), (0.0, 0, 64), (0.0, 1, 256), (0.001, 2, 64), (0.001, 0, 64)])
    res = s.run(reqs)
    assert sorted(r.rid for r in res) == [0, 1, 2, 3, 4]
    # universe 0's three requests ran one after another, warm-starting from the previous one
    starts = [e for e in eng.log if e[0] == "start" and e[2] == 0]
    assert [e[3] for e in starts] == [0, 20, 40]
    assert [e[4] for e in starts] == [False, True, True]
    # never two requests of one universe in the same chunk
    rid_u = {r.rid: r.universe for r in reqs}
    for e in eng.log:
        if e[0] == "advance":
            us = [rid_u[r] for r in e[1]]
            assert len(us) == len(set(us))
    # continuous batching: some chunk carried more than one request
    assert max(len(e[1]) for e in eng.log if e[0] == "advance") >= 2
    for r in res:
        assert r.latency >= 0 and r.done >= r.admitted >= r.arrival


def test_admission_respects_the_hbm_budget_and_rejects_oversize():
    clk = FakeClock()
    eng = FakeEngine(clk)
    one = footprint_bytes(256, 64, 256, "fp64")
    s = Scheduler(eng, P=64, generations=10, chunk=5, hbm_budget=int(1.5 * one), clock=clk)
    reqs = _reqs([(0.0, 0, 256), (0.0, 1, 256), (0.0, 2, 4096)])
    res = s.run(reqs)
    assert sorted(r.rid for r in res) == [0, 1]
    assert [r.rid for r in s.rejected] == [2]
    # the budget held only one 256-stock request at a time
    for e in eng.log:
        if e[0] == "advance":
            assert len(e[1]) == 1
    summ = s.summary()
    assert summ["requests"] == 2 and summ["rejected"] == 1 and summ["max_in_flight"] == 1


def test_stopped_requests_retire_early_and_the_next_window_continues_from_their_generation():
    clk = FakeClock()
    eng = FakeEngine(clk, stop_after={0: 12})
    s = Scheduler(eng, P=64, generations=40, chunk=5, hbm_budget=1 << 30, clock=clk)
    reqs = _reqs([(0.0, 0, 64), (0.0, 1, 64), (0.0, 0, 64)])
    res = {r.rid: r for r in s.run(reqs)}
    assert sorted(res) == [0, 1, 2]
    # request 0 stopped after 12 generations: it retired at the chunk boundary at 15
    adv0 = [e for e in eng.log if e[0] == "advance" and 0 in e[1]]
    assert len(adv0) == 3
    assert res[0].gen_end == 12
    # the universe's next window warm-started at generation 12; request 1 ran all 40
    starts = [e for e in eng.log if e[0] == "start" and e[2] == 0]
    assert [e[3] for e in starts] == [0, 12]
    assert res[1].gen_end == 40 and res[2].gen_end == 52


def test_resident_populations_count_against_the_budget_and_idle_ones_are_evicted():
    clk = FakeClock()
    eng = FakeEngine(clk)
    one = footprint_bytes(256, 64, 256, "fp64")
    res = resident_bytes(256, 64)
    budget = one + 3 * res                       # one request in flight plus three residents
    s = Scheduler(eng, P=64, generations=10, chunk=5, hbm_budget=budget, clock=clk)
    seen = []
    orig = eng.start

    def start(req, gen0, warm):
        seen.append(s.used)
        return orig(req, gen0, warm)

    eng.start = start
    # five universes in turn, then universe 0 again: its population was evicted by then
    reqs = _reqs([(0.001 * i, u, 256) for i, u in enumerate([0, 1, 2, 3, 4, 0])])
    out = {r.rid: r for r in s.run(reqs)}
    assert sorted(out) == list(range(6)) and not s.rejected
    assert max(seen) + one <= budget             # admission kept every moment within the budget
    assert s.used <= budget and len(s.resident) <= 3
    ev = [e[1] for e in eng.log if e[0] == "evict"]
    assert ev[:2] == [0, 1] and s.evictions == len(ev)   # least recently used first
    starts = [e for e in eng.log if e[0] == "start" and e[2] == 0]
    assert [e[4] for e in starts] == [False, False]      # universe 0 starts cold again ...
    assert [e[3] for e in starts] == [0, 10]             # ... at its next generation
    assert s.summary()["evictions"] == s.evictions
