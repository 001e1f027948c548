"""Benchmark: fitness evaluations/s and GA generations/s at N = 1024, BF16x2 vs FP64 form.

One step = the whole path for one correlation window of the precision-form
workload (N = 1024 stocks, T = 4096 returns, 32 planted clusters, P = 4096,
G = 300 generations): pga_correlate (+ BF16 split) -> pga_evolve (initial
population, 300 x [fitness, rank/statistics, breed], final fitness, one HIP
graph launch) -> pga_best. Inputs are synthetic (one-factor returns) and
resident in HBM before the timed region.

Prints one JSON line. `value` is fitness evaluations per second of the chosen
form over whole steps ((G + 1) * P per step), every individual through the
O(N^2) pair-sum of the form (cluster-pair route off); the FP64 form is timed
the same way for the speed-up. `roofline` is for the dominant kernel (the
pair-sum of the chosen form), its average duration measured with HIP events on
the launching stream. `route` repeats the steps with the library's default
cluster-pair route (individuals with few within-cluster pairs evaluated from
those pairs alone, exact FP64) and gives that kernel's own roofline.
`cpu_baseline` is the CPU oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

KIND_TAG = {0: "", 1: "p", 2: "l"}          # pair-sum MFMA kinds: register one-hot, packed, LDS table
PEAK_MFMA_BF16 = 2500.0          # TFLOP/s, dense bf16 MFMA (MI355X published)
PEAK_HBM = 8000.0                # GB/s
CU, SIMD, LANES, CLOCK = 256, 4, 16, 2.4e9
PEAK_ALU = CU * SIMD * LANES * CLOCK / 1e12   # Tops/s: one 32/64-bit VALU lane-op per lane per clock


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", choices=["bf16x2", "fp64"], default="bf16x2")
    ap.add_argument("--generations", type=int, default=300)
    ap.add_argument("--no-compare", action="store_true", help="skip timing the other form")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-route", action="store_true",
                    help="skip the measurements with the cluster-pair route (only the pair-sum route)")
    ap.add_argument("--calib-copy-mib", type=int, default=256,
                    help="size of the plain device copy run once for counter calibration")
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="length of the Poisson request stream of the serving run (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--batched-instances", type=int, default=256,
                    help="instances of the ragged batched run (0 = skip)")
    ap.add_argument("--paper-windows", type=int, default=1760,
                    help="18-stock windows of the run in the paper's own problem shape (0 = skip)")
    ap.add_argument("--tune-reps", type=int, default=5,
                    help="timed evaluations per pair-sum kernel variant in the autotuning pass")
    ap.add_argument("--variants", default="",
                    help="use these pair-sum kernel variants instead of autotuning, e.g. bf16x2=3,fp64=3")
    ap.add_argument("--tune-table", default="",
                    help="write the tuning table (every tuned shape) to this file at the end")
    ap.add_argument("--only", default="",
                    help="run only these parts (comma list of: main, batched, serving, paper) and print their JSON")
    return ap.parse_args()


def batched_run(n_inst, form, generations=200, reps=2, tune_table=None):
    """Ragged batched form: n_inst independent GA instances (N ~ U{32..512}, T = 1024,
    P = 512 each) advanced together by ONE pga_evolve call (one graph launch) per rep.
    The pair-sum variant for this batch (keyed by its largest N and total P) is chosen by
    timing short graph-replayed runs of every variant, and the tuning table is written to
    `tune_table` when given. One more run, eager with per-launch events, gives the kernel
    times of a generation and the launch gap of the graph replay."""
    import numpy as np
    import torch

    from paper_1403_4099_amd import pga, synth

    insts = []
    for i in range(n_inst):
        w = synth.config4_instance(i)
        R = torch.from_numpy(w.R).cuda()
        out = pga.correlate(R, split=(form == "bf16x2"))
        C, hi, lo = out if form == "bf16x2" else (out, None, None)
        insts.append(pga.make_instance(C, w.P, hi=hi, lo=lo, stats_rows=generations + 1, elites=w.elites,
                                       seed=w.seed, instance_id=i))
    max_n = max(I.N for I in insts)
    Ps = sum(I.P for I in insts)
    ctx = pga.Context()
    # ---- variant choice for this batch shape (short graph runs, best of 2 after a warm-up)
    tg = 20
    ms = {}
    for v in range(len(pga.variants(form))):
        pga.tune_set(form, max_n, Ps, v)
        if pga.tune_get(form, max_n, Ps) != v:          # does not fit this N
            continue
        ctx.evolve(insts, tg, form=form, init=True)
        best = float("inf")
        for _ in range(2):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ctx.evolve(insts, tg, form=form, init=True)
            torch.cuda.synchronize()
            best = min(best, time.perf_counter() - t0)
        ms[v] = 1e3 * best / tg
    vbest = min(ms, key=lambda v: (ms[v] > min(ms.values()) * 1.03, v))   # near-ties to the lower index
    pga.tune_set(form, max_n, Ps, vbest)
    saved = pga.tune_save(tune_table) if tune_table else None
    # ---- timed runs
    ctx.evolve(insts, generations, form=form, init=True)          # warm-up: captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.evolve(insts, generations, form=form, init=True)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    pairs = sum(I.P * I.N * (I.N - 1) / 2 for I in insts)
    # ---- kernel times of the same run (eager launches with events)
    pga.timing_enable(True)
    pga.timing_reset()
    ctx.evolve(insts, generations, form=form, init=True)
    torch.cuda.synchronize()
    kern = {}
    for kname in ("cluster_pairs", "nsmask", "pairsum_fp64", "pairsum_mfma", "finish", "rank", "breed", "init"):
        k_ms, n = pga.timing_read(kname)
        if n:
            kern[kname] = {"avg_us": 1e3 * k_ms / n, "launches": n}
    pga.timing_enable(False)
    per_gen_kernels = sum(v["avg_us"] * v["launches"] for k, v in kern.items() if k != "init") / (generations + 1)
    # ---- roofline of the cluster-pair step (route kernel + cluster-pair kernel, one launch each) on the
    # generation-0 population: a call with no generations initialises and evaluates it once
    pga.timing_enable(True)
    pga.timing_reset()
    for _ in range(3):
        ctx.evolve(insts, 0, form=form, init=True)
    torch.cuda.synchronize()
    ms_cp, n_cp = pga.timing_read("cluster_pairs")
    pga.timing_enable(False)
    t_cp = 1e-3 * ms_cp / n_cp
    frac_r = pga.route_get()
    byts, listed = 0.0, 0
    for I in insts:
        wp = within_pairs(I.pop)
        lim = I.N * (I.N - 1) // 2 if I.N <= 64 else np.floor(frac_r * 0.5 * I.N * (I.N - 1))
        on = (wp <= lim) if I.N <= 2048 else np.zeros(len(wp), dtype=bool)
        listed += int(on.sum())
        byts += I.P * 4.0 * I.N + 8.0 * float(on.sum()) + 8.0 * float(wp[on].sum()) + 8.0 * I.N
    ach = byts / t_cp / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM, "unit": "GB/s", "frac": ach / PEAK_HBM,
            "traffic": None, "kernel": "k_route + k_sparse_wave", "avg_launch_us": 1e6 * t_cp,
            "listed_share": listed / Ps,
            "work_per_launch": "every individual's labels (4N B), and for those within the pair limit the "
                               "fitness (8 B) and their within-cluster C entries (8 B each); each instance's "
                               "diagonal once; generation-0 populations"}
    ctx.close()
    return {"instances": n_inst, "form": form, "generations": generations,
            "seconds_per_run": dt, "gens_per_s": generations / dt,
            "fitness_evals_per_s": Ps * (generations + 1) / dt,
            "pair_visits_per_s": pairs * (generations + 1) / dt,
            "sum_N": int(sum(I.N for I in insts)), "max_N": max_n, "sum_P": Ps,
            "variant": {"chosen": vbest, "ms_per_generation": {str(k): round(v, 4) for k, v in ms.items()},
                        "table_entries_saved": saved},
            "kernels_us": kern,
            "generation_us": {"graph_wall": 1e6 * dt / generations, "eager_kernel_sum": per_gen_kernels},
            "roofline_cluster_pairs": roof,
            "workload": "256 instances, N ~ U{32..512}, T=1024, 2-12 planted clusters, P=512, G=200"}


def paper_shape_run(form, n_windows=1760, T=1800, generations=400, singles=12):
    """The paper's own problem shape (Section 4.2, Tables 3 and 4): one 18-stock correlation matrix per
    window, population 1000, at most 400 generations with the termination test (stall 50 generations,
    tolerance 1e-5) and 10 elites. Synthetic windows (three planted clusters of 8, 6 and 4 stocks,
    loadings U[0.3, 0.7], T = 1800 returns, about the points per stock of the paper's test set) stand
    in for its 1760 JSE matrices. (a) windows one at a time, each correlate + evolve + best
    synchronised, as the paper clustered them; (b) all windows as one batch (one evolve call). Context
    for the paper's Table 4 medians (0.80 s per matrix on a GTX Titan Black, 1.39 s on a Tesla C2050),
    not a like-for-like comparison: other hardware, other data, and the paper's own crossover."""
    import numpy as np
    import torch

    from paper_1403_4099_amd import pga, synth

    rng = np.random.default_rng(7)
    Rs = []
    for _ in range(n_windows):
        R, _ = synth.one_factor_returns([8, 6, 4], rng.uniform(0.3, 0.7, size=3), 0, T, rng)
        Rs.append(torch.from_numpy(R).cuda())
    split = form == "bf16x2"

    def corr(R):
        out = pga.correlate(R, split=split)
        return out if split else (out, None, None)

    def inst(C, hi, lo, i):
        return pga.make_instance(C, 1000, hi=hi, lo=lo, elites=10, seed=11, instance_id=i, stall_gens=50,
                                 tol=1e-5)

    ctx = pga.Context()
    # (a) one window at a time (the first two calls capture the graph and are left out)
    times, gens = [], []
    for w in range(singles):
        C, hi, lo = corr(Rs[w])
        I = inst(C, hi, lo, w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        C, hi, lo = corr(Rs[w])
        I.C, I.hi, I.lo = C, hi, lo
        ctx.evolve([I], generations, form=form, init=True)
        pga.best(I.fitness, I.pop)                               # synchronises
        times.append(time.perf_counter() - t0)
        gens.append(I.term_state()["gens"])
    # (b) every window in one batch: the windows' correlations, one evolve call, every best labeling
    cs = [corr(R) for R in Rs]
    batch = [inst(C, hi, lo, i) for i, (C, hi, lo) in enumerate(cs)]
    ctx.evolve(batch, generations, form=form, init=True)        # warm-up: captures the graph
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cs = [corr(R) for R in Rs]
    for I, (C, hi, lo) in zip(batch, cs):
        I.C, I.hi, I.lo = C, hi, lo
    ctx.evolve(batch, generations, form=form, init=True)
    for I in batch:
        pga.best(I.fitness, I.pop)
    dt = time.perf_counter() - t0
    bgens = [I.term_state()["gens"] for I in batch]
    ctx.close()
    single = float(np.median(times[2:]))
    return {"form": form, "windows": n_windows,
            "seconds_per_matrix_one_at_a_time": single,
            "generations_one_at_a_time_mean": float(np.mean(gens)),
            "matrices_per_s_batched": n_windows / dt, "seconds_batched": dt,
            "generations_batched_mean": float(np.mean(bgens)), "generations_batched_max": int(max(bgens)),
            "paper_table4_seconds_per_matrix": {"GTX Titan Black (CUDA)": 0.80, "Tesla C2050 (CUDA)": 1.39},
            "workload": "N=18, T=1800, planted 8/6/4, P=1000, <=400 generations, stall 50, tol 1e-5, 10 elites, "
                        "tournament selection and uniform crossover (the paper: its knowledge-based crossover)"}


def serving_run(seconds, rate, form, stall_gens=0, tol=1e-5, eager=False):
    """Continuous-batching run over a Poisson stream of correlation windows (N in {64, 256, 1024}
    at 6:3:1, T = 390, P = 1024 resident and warm-started per universe, up to 100 generations per
    request in chunks of 10, 8 GiB admission budget). Windows are staged in HBM beforehand. With
    stall_gens > 0 a request also ends when its GA's termination test fires (Table 3)."""
    import numpy as np
    import torch

    from paper_1403_4099_amd import synth
    from paper_1403_4099_amd.serve import GpuEngine, Request, Scheduler

    _, stream = synth.serving_stream(duration=seconds, rate=rate, seed=4)
    reqs = [Request(i, u, t, torch.from_numpy(R).cuda(), R.shape[0], R.shape[1])
            for i, (t, u, R) in enumerate(stream)]
    torch.cuda.synchronize()
    eng = GpuEngine(P=1024, form=form, stall_gens=stall_gens, tol=tol, eager=eager)
    sch = Scheduler(eng, P=1024, generations=100, chunk=10, hbm_budget=8 << 30, form=form)
    res = sch.run(reqs)
    out = sch.summary()
    out.update({"offered_rate_per_s": rate, "stream_seconds": seconds, "form": form,
                "launch": "eager" if eager else f"HIP graphs ({eng.ctx.graphs()} cached at the end)",
                "termination": {"stall_gens": stall_gens, "tol": tol} if stall_gens else None,
                "workload": "Poisson windows, N in {64,256,1024} 6:3:1 over 16 universes, T=390, "
                            "P=1024, up to 100 generations, 5% drift per window"})
    if stall_gens:
        out["mean_generations_per_request"] = float(np.mean(_gens_per_request(res)))
    return out


def _gens_per_request(results):
    """Generations each request ran (the difference of its universe's generation counter)."""
    last = {}
    out = []
    for r in sorted(results, key=lambda r: r.done):
        out.append(r.gen_end - last.get(r.universe, 0))
        last[r.universe] = r.gen_end
    return out


# ---------------------------------------------------------------- launch geometry (issued work)
def mfma_issued_flops(pop, B: int = 8, kind: int = 0) -> float:
    """MFMA flops the BF16x2 pair-sum kernel issues for one launch on population `pop` (P x N,
    on the device; every individual through the pair-sum), two MFMAs (hi, lo) of 16 x 16 x 32 x 2
    flops per column group and 32-row chunk up to the 16-stock tile's diagonal. Column kernels
    (kind 0, register one-hot; kind 2, LDS-table one-hot): one group per individual of each batch
    of B. Packed kernel (kind 1): ceil(sum_b K_b / 16) groups per tile and batch, run in pairs
    (K_b: labels of the tile held by >= 2 stocks of individual b)."""
    import torch
    P_, N_ = pop.shape
    if kind != 1:
        n_tiles = -(-N_ // 16)
        chunks = sum(-(-min(16 * w + 16, N_) // 32) for w in range(n_tiles))
        return float(chunks * 2 * B * -(-P_ // B)) * 16 * 16 * 32 * 2
    pad = (-N_) % 16
    lab = pop.long()
    cnt = torch.zeros((P_, N_), dtype=torch.int32, device=pop.device)
    cnt.scatter_add_(1, lab, torch.ones_like(pop))
    key = torch.where(torch.gather(cnt, 1, lab) >= 2, lab, torch.full_like(lab, -1))
    if pad:
        key = torch.cat([key, torch.full((P_, pad), -1, dtype=key.dtype, device=key.device)], dim=1)
    t = key.view(P_, -1, 16).sort(dim=2).values
    first = torch.ones_like(t, dtype=torch.bool)
    first[..., 1:] = t[..., 1:] != t[..., :-1]
    k = (first & (t >= 0)).sum(dim=2)                               # K per (individual, tile)
    bpad = (-P_) % B
    if bpad:
        k = torch.cat([k, torch.zeros((bpad, k.shape[1]), dtype=k.dtype, device=k.device)], dim=0)
    s = k.view(-1, B, k.shape[1]).sum(dim=1)                        # columns per (batch, tile)
    nq = (s + 15) // 16
    nq2 = (nq + 1) // 2 * 2
    tiles = torch.arange(k.shape[1], device=pop.device)
    chunks = (torch.clamp(tiles * 16 + 16, max=N_) + 31) // 32      # chunks up to the tile's diagonal
    mfmas = (nq2 * chunks[None, :]).sum().item() * 2
    return float(mfmas) * 16 * 16 * 32 * 2


def kbar_tiles(pop) -> float:
    """Mean one-hot width of the compacted contraction: over every individual and every tile of
    16 consecutive stocks, the number of distinct labels in the tile held by at least two stocks
    of the individual (singletons need no column). Computed with torch on the device."""
    import torch
    P_, N_ = pop.shape
    pad = (-N_) % 16
    lab = pop.long()
    cnt = torch.zeros((P_, N_), dtype=torch.int32, device=pop.device)
    cnt.scatter_add_(1, lab, torch.ones_like(pop))
    ns = torch.gather(cnt, 1, lab)                                # n_s of each stock's label
    key = torch.where(ns >= 2, lab, torch.full_like(lab, -1))
    if pad:
        key = torch.cat([key, torch.full((P_, pad), -1, dtype=key.dtype, device=key.device)], dim=1)
    t = key.view(P_, -1, 16).sort(dim=2).values
    first = torch.ones_like(t, dtype=torch.bool)
    first[..., 1:] = t[..., 1:] != t[..., :-1]
    k = (first & (t >= 0)).sum(dim=2)
    return float(k.double().mean())


def method_flops_bf16x2(N: int, P: int, kbar: float) -> float:
    """Flops of the compacted one-hot contraction per launch: hi and lo, 2 flops per
    multiply-add, N^2 / 2 (the triangle i < j) times the mean one-hot width kbar, P individuals."""
    return 2.0 * N * N * kbar * P


def pair_visits(N: int, P: int) -> float:
    """Unordered pairs i < j times individuals: the work the method must do per population evaluation."""
    return float(N) * (N - 1) / 2 * P


def within_pairs(pop) -> "np.ndarray":
    """sum_s n_s (n_s - 1) / 2 of every row of a population (host)."""
    import numpy as np
    a = pop.cpu().numpy() if hasattr(pop, "cpu") else pop
    N = a.shape[1]
    out = np.empty(a.shape[0], dtype=np.int64)
    for r in range(a.shape[0]):
        n = np.bincount(a[r], minlength=N).astype(np.int64)
        out[r] = int((n * (n - 1) // 2).sum())
    return out


def source_sha(path):
    """Hash of a kernel source together with the shared header that fixes its tile geometry."""
    h = hashlib.sha256()
    for p in (path, os.path.join(os.path.dirname(path), "pga_internal.hpp")):
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel_src: str, N: int, P: int, variant: int):
    """HBM bytes per launch from the committed counter summary, if it was taken on this kernel source
    and kernel variant."""
    fn = os.path.join(ROOT, "profiles", "traffic_per_launch.txt")
    if not os.path.exists(fn):
        return None
    sha = source_sha(kernel_src)
    for line in open(fn):
        f = line.split()
        if (len(f) >= 6 and not line.startswith("#") and f[0] == sha and int(f[1]) == N and int(f[2]) == P
                and int(f[3]) == variant):
            return float(f[4]) + float(f[5])
    return None


# ---------------------------------------------------------------- CPU baseline (oracle)
def _cpu_info():
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)), "model": None}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def cpu_baseline(w, P, seed, gens=3, gpu_check=None):
    """The oracle, unchanged, on the host cores: `gens` generations of the workload from its initial
    population (fitness of the whole population split into row blocks evaluated by concurrent calls
    into the oracle, each call single-threaded C that releases the GIL; then one breed step).
    Threads: the CPUs this process may run on, at most 16 (the CPU share of a one-GPU job).
    gpu_check(C, pop0, f0) may compare the GPU's results with the oracle's on the same inputs."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle as O

    threads = max(1, min(16, len(os.sched_getaffinity(0))))
    t0 = time.perf_counter()
    C = O.correlate(w.R)
    t_corr = time.perf_counter() - t0
    pop = O.init_pop(w.N, P, seed=seed)
    pop0, f0 = pop, None
    t0 = time.perf_counter()
    O.fitness(C, pop[: max(1, P // threads)])
    t_one = time.perf_counter() - t0
    blocks = np.array_split(np.arange(P), threads)
    t_fit = t_breed = 0.0
    with ThreadPoolExecutor(threads) as ex:
        for g in range(gens):
            t0 = time.perf_counter()
            parts = list(ex.map(lambda ix, pop=pop: O.fitness(C, pop[ix]), blocks))
            t_fit += time.perf_counter() - t0
            f = np.concatenate(parts)
            if g == 0:
                f0 = f
            t0 = time.perf_counter()
            pop = O.breed(pop, f, E=2, seed=seed, gen=g)
            t_breed += time.perf_counter() - t0
    evals_per_s = gens * P / (t_fit + t_breed)
    ci = _cpu_info()
    out = {
        "value": evals_per_s, "unit": "fitness evals/s", "cores": threads, "kind": "oracle",
        "sample": (f"{gens} generations of the N={w.N}, P={P} workload on the CPU oracle with {threads} "
                   f"threads ({ci['affinity']} CPUs allotted of nproc {ci['nproc']}, {ci['model']}): fitness "
                   f"{t_fit:.2f} s + breed {t_breed:.2f} s; one thread alone: "
                   f"{max(1, P // threads) / t_one:.0f} evals/s; the window's correlation took "
                   f"{t_corr:.2f} s and is not in the rate"),
        "gens_per_s": gens / (t_fit + t_breed),
        "correlate_s": t_corr,
        "cpu": ci,
    }
    if gpu_check is not None:
        out["gpu_vs_oracle"] = gpu_check(C, pop0, f0, ex_threads=threads)
    return out


def route_section(args, forms, results, insts, timed, step, pop0, route_default, C, hi, lo, N, P, G):
    """The cluster-pair route at the library's default limit: the same steps, its kernels, and
    pga_fitness calls on the random and on the route run's final population."""
    import numpy as np
    import torch

    from paper_1403_4099_amd import pga
    pga.route_set(route_default)
    lim = int(np.floor(route_default * 0.5 * N * (N - 1)))
    route = {"limit_frac": route_default, "limit_pairs": lim,
             "rule": "an individual with at most limit_pairs pairs inside its clusters (N <= 2048) is evaluated "
                     "from those pairs (exact FP64); the others by the pair-sum of the form", "steps": {}}
    for form in forms:
        wall, ev, (lab, fbest, idx) = timed(form, args.steps, args.warmup)
        route["steps"][form] = {"fitness_evals_per_s": (G + 1) * P * args.steps / wall,
                                "gens_per_s": G * args.steps / wall, "ms_per_step": 1e3 * wall / args.steps,
                                "speedup_vs_pairsum_only": results[form]["wall_s"] / wall, "best_Lc": fbest}
        print(f"[bench] route {form}: {route['steps'][form]}", file=sys.stderr, flush=True)
    pga.timing_enable(True)
    rk = {}
    for form in forms:
        pga.timing_reset()
        step(form)
        torch.cuda.synchronize()
        for kname in ("cluster_pairs", "pairsum_fp64", "pairsum_mfma", "finish", "rank", "breed"):
            ms, n = pga.timing_read(kname)
            if n:
                rk.setdefault(form, {})[kname] = {"avg_us": 1e3 * ms / n, "launches": n}
    pga.timing_enable(False)
    route["kernels_us"] = rk
    wp0 = within_pairs(pop0)
    wpf = within_pairs(insts[args.form].pop)
    route["population_pairs"] = {"random_mean": float(wp0.mean()), "final_mean": float(wpf.mean()),
                                 "final_share_within_limit": float((wpf <= lim).mean())}
    route["fitness_call"] = {}
    t_route = None
    for form in forms:
        for tag, pop in (("random", pop0), ("final", insts[form].pop)):
            for _ in range(3):
                pga.fitness(C, pop, form, hi=hi, lo=lo)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(20):
                pga.fitness(C, pop, form, hi=hi, lo=lo)
            e1.record()
            torch.cuda.synchronize()
            t_call = e0.elapsed_time(e1) * 1e-3 / 20
            pga.timing_enable(True)
            pga.timing_reset()
            for _ in range(5):
                pga.fitness(C, pop, form, hi=hi, lo=lo)
            torch.cuda.synchronize()
            ms, n = pga.timing_read("cluster_pairs")
            pga.timing_enable(False)
            t_k = 1e-3 * ms / n
            route["fitness_call"].setdefault(form, {})[tag] = {
                "fitness_call_us": 1e6 * t_call, "fitness_evals_per_s": P / t_call,
                "cluster_pairs_us": 1e6 * t_k}
            if form == args.form and tag == "random":
                t_route = t_k
    # algorithmic bytes of one launch on the random population: labels, the C entries of the
    # within-cluster pairs, the fitness, and the diagonal once
    byts = P * (4.0 * N + 8.0) + 8.0 * float(wp0.sum()) + 8.0 * N
    ach = byts / t_route / 1e9
    route["roofline"] = {"bound": "hbm", "achieved": ach, "peak": PEAK_HBM, "unit": "GB/s", "frac": ach / PEAK_HBM,
                         "traffic": recorded_traffic(os.path.join(ROOT, "paper_1403_4099_amd", "csrc",
                                                                  "k_fitness.hip"), N, P, -1),
                         "kernel": "k_sparse", "avg_launch_us": 1e6 * t_route,
                         "work_per_launch": "labels (4N B), within-cluster C entries (8 B each, "
                                            f"{float(wp0.mean()):.0f} pairs per individual), fitness, diagonal "
                                            "once, on the random generation-0 population"}
    return route


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU sharding is a "
              f"design note and is not run here", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1403_4099_amd import pga, synth

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if args.only:
        # one part alone (for profiling it): its JSON object on one line, no headline
        parts = set(args.only.split(","))
        out = {}
        if "batched" in parts:
            out["batched"] = batched_run(args.batched_instances or 256, args.form,
                                         tune_table=args.tune_table or None)
        if "serving" in parts:
            out["serving"] = serving_run(args.serve_seconds or 5.0, args.serve_rate, args.form)
        if "paper" in parts:
            out["paper_shape"] = paper_shape_run(args.form, args.paper_windows or 1760)
        print(json.dumps(out))
        return
    route_default = pga.route_get()
    pga.route_set(0.0)          # headline: every individual through the pair-sum of its form
    w = synth.config3()
    N, T, P, G = w.N, w.T, w.P, args.generations
    R = torch.from_numpy(w.R).to(dev)
    ld = pga.split_ld(N)
    C = torch.empty((N, N), dtype=torch.float64, device=dev)
    hi = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    lo = torch.empty((ld, ld), dtype=torch.int16, device=dev)
    status = pga.new_status(dev)
    cws = torch.empty(pga.load().pga_correlate_ws_bytes(N), dtype=torch.uint8, device=dev)
    ctx = pga.Context()
    insts = {}

    def step(form):
        L = pga.load()
        stream = pga._stream()
        split = form == "bf16x2"
        rc = L.pga_correlate(pga._ptr(R), N, T, R.stride(0), pga._ptr(C), pga._ptr(hi) if split else None,
                             pga._ptr(lo) if split else None, pga._ptr(status), pga._ptr(cws), cws.numel(),
                             stream)
        pga._check(rc, "pga_correlate")
        I = insts.get(form)
        if I is None:
            I = pga.make_instance(C, P, hi=hi, lo=lo, stats_rows=G + 1, elites=w.elites, seed=w.seed)
            insts[form] = I
        ctx.evolve([I], G, form=form, init=True, status=status)
        return pga.best(I.fitness, I.pop)

    def timed(form, steps, warmup):
        for _ in range(warmup):
            step(form)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        res = None
        for _ in range(steps):
            res = step(form)
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return wall, e0.elapsed_time(e1) / 1e3, res

    forms = [args.form] + ([] if args.no_compare else [f for f in ("bf16x2", "fp64") if f != args.form])

    # ---- autotune the pair-sum kernel of each form on this shape (random labelings of the workload)
    L = pga.load()
    rc = L.pga_correlate(pga._ptr(R), N, T, R.stride(0), pga._ptr(C), pga._ptr(hi), pga._ptr(lo),
                         pga._ptr(status), pga._ptr(cws), cws.numel(), pga._stream())
    pga._check(rc, "pga_correlate")
    pop_tune = torch.from_numpy(synth.random_labelings(P, N, seed=7)).to(dev)
    tuned = {}
    fixed = dict(kv.split("=") for kv in args.variants.split(",") if kv)
    for form in forms:
        if form in fixed:
            v, ms = int(fixed[form]), None
            pga.tune_set(form, N, P, v)
        else:
            v, ms = pga.tune(C, pop_tune, form, hi=hi, lo=lo, reps=args.tune_reps)
        tuned[form] = {"variant": v, "individuals_per_group": pga.variants(form)[v][0],
                       "xcd_order": pga.variants(form)[v][1], "kind": pga.variants(form)[v][2],
                       "ms_per_variant": None if ms is None else
                       {f"{a}x{b}{KIND_TAG[c]}": round(m, 4) for (a, b, c), m in zip(pga.variants(form), ms)}}
        print(f"[bench] {'variant' if ms is None else 'autotune'} {form}: {tuned[form]}", file=sys.stderr,
              flush=True)
    del pop_tune

    results = {}
    for form in forms:
        wall, ev, (lab, fbest, idx) = timed(form, args.steps, args.warmup)
        results[form] = {"wall_s": wall, "event_s": ev, "best": fbest, "labels": lab,
                         "clusters": int(len(set(lab.tolist())))}
        print(f"[bench] {form}: {args.steps} steps in {wall:.3f} s (events {ev:.3f} s), best L_c {fbest:.6f}",
              file=sys.stderr, flush=True)

    # ---- kernel timing (HIP events around each launch, eager launches), same workload
    pga.timing_enable(True)
    kern = {}
    for form in forms:
        pga.timing_reset()
        step(form)
        torch.cuda.synchronize()
        for k in ("pairsum_fp64", "pairsum_mfma", "finish", "rank", "breed", "correlate", "split", "init"):
            ms, n = pga.timing_read(k)
            if n:
                kern.setdefault(form, {})[k] = {"avg_us": 1e3 * ms / n, "launches": n}
    pga.timing_enable(False)

    # ---- mean one-hot width (compacted, per 16-stock tile) of every population the timed generation
    # loop evaluates: the same run replayed one generation per call (identical trajectory)
    kb_loop = {}
    for form in forms:
        if form != "bf16x2":
            continue
        I = insts[form]
        B, pk = tuned[form]["individuals_per_group"], tuned[form]["kind"]
        ctx.evolve([I], 0, form=form, init=True)
        kbs = [kbar_tiles(I.pop)]
        iss = [mfma_issued_flops(I.pop, B, pk)]
        for g in range(G):
            I.gen0 = g
            ctx.evolve([I], 1, form=form)
            kbs.append(kbar_tiles(I.pop))
            iss.append(mfma_issued_flops(I.pop, B, pk))
        I.gen0 = 0
        kb_loop[form] = {"mean": float(np.mean(kbs)), "generation_0": kbs[0], "final": kbs[-1],
                         "issued_flops_mean": float(np.mean(iss))}
        print(f"[bench] one-hot width per 16-stock tile over the loop ({form}): {kb_loop[form]}",
              file=sys.stderr, flush=True)

    # ---- precision: BF16x2 vs FP64 fitness on the same populations
    prec = {}
    pop0 = torch.from_numpy(synth.random_labelings(P, N, seed=123)).to(dev)
    if "bf16x2" in results and "fp64" in results:
        def both(pop):
            f64 = pga.fitness(C, pop, "fp64")
            fbf = pga.fitness(C, pop, "bf16x2", hi=hi, lo=lo)
            rel = float(((fbf - f64).abs() / f64.abs().clamp_min(1e-300)).max())
            l64, _, _ = pga.best(f64, pop)
            lbf, _, _ = pga.best(fbf, pop)
            return rel, bool(np.array_equal(l64, lbf))
        rel_final, same_final = both(insts["bf16x2"].pop)
        rel_f64run, same_f64run = both(insts["fp64"].pop)
        rel_init, same_init = both(pop0)
        prec = {"max_rel_err_converged_pop": max(rel_final, rel_f64run), "max_rel_err_random_pop": rel_init,
                "same_population_identical_best": same_final and same_f64run,
                "ga_runs_identical_best": bool(np.array_equal(results["bf16x2"]["labels"],
                                                              results["fp64"]["labels"])),
                "best_Lc": {f: results[f]["best"] for f in results},
                "note": "same_population: each GA run's final population evaluated by both forms, same argmax "
                        "labeling; ga_runs: the two forms' separate GA runs (trajectories part at near-ties)"}

    # ---- pga_fitness on a resident population: median of 20 timed calls after 3 warm-ups (HIP
    # events on the calling stream, calls back to back), at the random (generation 0) and converged
    # populations, with
    # the pair-sum kernel's own time (library timing, same calls) and the population's mean K
    def kbar(pop):
        srt = pop.sort(dim=1).values
        return float(((srt[:, 1:] != srt[:, :-1]).sum(dim=1) + 1).double().mean())
    by_pop = {}
    for form in forms:
        kname = "pairsum_mfma" if form == "bf16x2" else "pairsum_fp64"
        for tag, pop in (("random", pop0), ("converged", insts[form].pop)):
            for _ in range(3):
                pga.fitness(C, pop, form, hi=hi, lo=lo)
            # back to back, one synchronisation at the end: the GPU stays busy as in a serving loop
            # (with a host round trip after every call its clock does not settle at the loaded rate)
            evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                   for _ in range(20)]
            for e0, e1 in evs:
                e0.record()
                pga.fitness(C, pop, form, hi=hi, lo=lo)
                e1.record()
            torch.cuda.synchronize()
            calls = [e0.elapsed_time(e1) * 1e-3 for e0, e1 in evs]
            pga.timing_enable(True)
            pga.timing_reset()
            for _ in range(5):
                pga.fitness(C, pop, form, hi=hi, lo=lo)
            torch.cuda.synchronize()
            ms, n = pga.timing_read(kname)
            pga.timing_enable(False)
            t_call = float(np.median(calls))
            t_ps = 1e-3 * ms / n
            entry = {"fitness_call_us": 1e6 * t_call, "fitness_evals_per_s": P / t_call,
                     "pair_equivalent_per_s": pair_visits(N, P) / t_call,
                     "pairsum_us": 1e6 * t_ps, "mean_K": kbar(pop)}
            if form == "bf16x2":
                kt = kbar_tiles(pop)
                entry["kbar_tile"] = kt
                entry["pairsum_roofline_frac"] = method_flops_bf16x2(N, P, kt) / t_ps / 1e12 / PEAK_MFMA_BF16
                entry["pairsum_issued_frac"] = (mfma_issued_flops(pop, tuned[form]["individuals_per_group"],
                                                                  tuned[form]["kind"])
                                                / t_ps / 1e12 / PEAK_MFMA_BF16)
            else:
                entry["pairsum_roofline_frac"] = 2 * pair_visits(N, P) / t_ps / 1e12 / PEAK_ALU
            by_pop.setdefault(form, {})[tag] = entry

    # ---- the generation loop: wall time per generation minus the kernels it runs
    loop = {}
    for f in results:
        kk = kern.get(f, {})
        per_gen_us = 1e6 * results[f]["wall_s"] / (args.steps * G)
        ksum = sum(kk[k]["avg_us"] for k in ("pairsum_mfma" if f == "bf16x2" else "pairsum_fp64", "finish",
                                              "rank", "breed") if k in kk)
        loop[f] = {"wall_us_per_generation": per_gen_us, "kernel_us_per_generation": ksum,
                   "note": "wall includes correlate, split, init and best once per step; kernel times are "
                           "eager launches with events, slightly above their graph-replay durations"}

    # ---- the cluster-pair route at the library's default limit: the same steps, its kernels, and
    # pga_fitness calls on the random and on the route run's final population
    route = None
    if not args.no_route:
        route = route_section(args, forms, results, insts, timed, step, pop0, route_default, C, hi, lo, N, P, G)

    # ---- calibration copy for the HBM counters (plain device-to-device copy of known size), timed
    # as the measured HBM ceiling (read + write bytes over the best of 5 copies), and the measured
    # bf16 MFMA ceiling (the library's register-operand MFMA loop)
    nb = args.calib_copy_mib << 20
    a = torch.empty(nb, dtype=torch.uint8, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    t_copy = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        t_copy = min(t_copy, e0.elapsed_time(e1) * 1e-3)
    del a, b
    fp64_tf = pga.peak_fp64()
    mix = {k: round(v, 1) for k, v in pga.pipe_mix(n_workgroups=4096, iters=2000).items()}
    peaks = {"hbm_copy_GBps": 2 * nb / t_copy / 1e9, "mfma_bf16_TFLOPs": pga.peak_mfma_bf16(),
             "fp64_fma_TFLOPs": fp64_tf, "alu_lane_ops_Tops": fp64_tf / 2.0,
             "pipe_mix_cycles_per_round": mix,
             "pipe_mix_note": ("cycles per round per wave on one SIMD (pga_pipe_mix): a round is 4 MFMAs, or "
                               "one individual's register one-hot (8 VALU ops), or 2 LDS 16-byte reads; "
                               "'a+b' both in each wave, 'a|b' on alternate waves"),
             "published": {"hbm_GBps": 8000.0, "mfma_bf16_TFLOPs": PEAK_MFMA_BF16, "fp64_TFLOPs": 78.6,
                           "alu_Tops": PEAK_ALU},
             "note": "sustained rates measured on this GPU (HBM: device copy; MFMA: register-operand "
                     "16x16x32 bf16 loop; FP64: register-operand v_fma_f64 loop, one lane-op = one FMA); "
                     "roofline.frac uses the published peak"}

    form = args.form
    res = results[form]
    evals = (G + 1) * P * args.steps
    value = evals / res["wall_s"]
    k = kern[form]["pairsum_mfma" if form == "bf16x2" else "pairsum_fp64"]
    t_launch = k["avg_us"] * 1e-6
    src = os.path.join(ROOT, "paper_1403_4099_amd", "csrc", "k_mfma.hip" if form == "bf16x2" else "k_fitness.hip")
    if form == "bf16x2":
        kb = kb_loop[form]["mean"]
        achieved = method_flops_bf16x2(N, P, kb) / t_launch / 1e12
        issued = kb_loop[form]["issued_flops_mean"] / t_launch / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": PEAK_MFMA_BF16, "unit": "TFLOP/s",
                "frac": achieved / PEAK_MFMA_BF16, "traffic": recorded_traffic(src, N, P, tuned[form]["variant"]),
                "kernel": "k_pairsum_mfma", "avg_launch_us": k["avg_us"],
                "work_per_launch": (f"compacted one-hot contraction 2 * N^2 * Kbar * P flops (hi and lo, the "
                                    f"triangle i < j, Kbar = {kb:.2f} distinct labels held by >= 2 stocks per "
                                    f"16-stock tile, mean over the {G + 1} populations the loop evaluates)"),
                "kbar": kb_loop[form],
                "issued": {"achieved": issued, "frac": issued / PEAK_MFMA_BF16,
                           "work_per_launch": "issued v_mfma_f32_16x16x32_bf16 flops (hi and lo; one column per "
                                              "stock, or packed column groups of 16 run in pairs, as the tuned "
                                              "variant's kind has it), mean over the loop's populations"}}
    else:
        achieved = 2 * pair_visits(N, P) / t_launch / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU, "unit": "Tops/s",
                "frac": achieved / PEAK_ALU, "traffic": recorded_traffic(src, N, P, tuned[form]["variant"]),
                "kernel": "k_pairsum_fp64", "avg_launch_us": k["avg_us"],
                "work_per_launch": "2 ops (label compare, FP64 add) per unordered pair per individual"}
    if form == "bf16x2":
        roof["frac_of_measured_peak"] = achieved / peaks["mfma_bf16_TFLOPs"]
    else:
        roof["frac_of_measured_peak"] = achieved / peaks["alu_lane_ops_Tops"]
    other = {}
    for f in results:
        if f == form:
            continue
        kk = kern[f]["pairsum_mfma" if f == "bf16x2" else "pairsum_fp64"]
        other[f] = {"fitness_evals_per_s": (G + 1) * P * args.steps / results[f]["wall_s"],
                    "gens_per_s": G * args.steps / results[f]["wall_s"],
                    "ms_per_step": 1e3 * results[f]["wall_s"] / args.steps,
                    "pairsum_avg_us": kk["avg_us"],
                    "pairsum_alu_frac": (2 * pair_visits(N, P) / (kk["avg_us"] * 1e-6) / 1e12) / PEAK_ALU
                    if f == "fp64" else None}
    line = {
        "metric": "fitness evals/s + GA generations/s, BF16-split vs FP64 form at N=1024",
        "value": value,
        "unit": "fitness evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * res["wall_s"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16x2+f64" if form == "bf16x2" else "f64",
        "data": "synthetic",
        "config": {"workload": f"precision-form N={N} T={T} P={P} G={G}, 32 planted geometric clusters",
                   "form": form, "N": N, "T": T, "P": P, "generations": G, "parallelism": "single GPU",
                   "route": "off: every individual through the pair-sum of the form (see route)"},
        "gens_per_s": G * args.steps / res["wall_s"],
        "pair_visits_per_s": pair_visits(N, P) * (G + 1) * args.steps / res["wall_s"],
        "speedup_vs_fp64": (results["fp64"]["wall_s"] / res["wall_s"]) if (form == "bf16x2" and "fp64" in results) else None,
        "other_forms": other,
        "kernels_us": kern,
        "precision": prec,
        "fitness_call": by_pop,
        "generation_loop": loop,
        "peaks_measured": peaks,
        "autotune": tuned,
        "roofline": roof,
    }
    line["route"] = route
    pga.route_set(route_default)
    # the batched and serving runs use the library's default route
    if args.batched_instances > 0:
        line["batched"] = batched_run(args.batched_instances, form, tune_table=args.tune_table or None)
        line["batched"]["route_frac"] = route_default
        print(f"[bench] batched: {line['batched']}", file=sys.stderr, flush=True)
    if args.serve_seconds > 0:
        line["serving"] = serving_run(args.serve_seconds, args.serve_rate, form)
        line["serving"]["route_frac"] = route_default
        print(f"[bench] serving: {line['serving']}", file=sys.stderr, flush=True)
        se = serving_run(args.serve_seconds, args.serve_rate, form, eager=True)
        line["serving"]["eager_launches"] = {k: se[k] for k in ("p50_ms", "p99_ms", "requests_per_s", "chunks")}
        line["serving_with_termination"] = serving_run(args.serve_seconds, args.serve_rate, form,
                                                       stall_gens=10, tol=1e-5)
        line["serving_with_termination"]["route_frac"] = route_default
        print(f"[bench] serving with termination: {line['serving_with_termination']}", file=sys.stderr,
              flush=True)
    if args.paper_windows > 0:
        line["paper_shape"] = paper_shape_run(form, args.paper_windows)
        line["paper_shape"]["route_frac"] = route_default
        print(f"[bench] paper shape: {line['paper_shape']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        pga.route_set(0.0)      # the precision statement is for the pair-sum of the form

        def gpu_check(C_o, pop0_o, f0_o, ex_threads):
            """BF16x2 fitness (pair-sum route) against the FP64 oracle, per result, on the initial
            population and on the BF16x2 GA run's final population; and whether both pick the same
            best labeling."""
            from concurrent.futures import ThreadPoolExecutor

            import oracle as O
            out = {}
            with ThreadPoolExecutor(ex_threads) as ex:
                for tag, popn in (("random_generation_0", pop0_o),
                                  ("ga_final_population", insts["bf16x2"].pop.cpu().numpy()
                                   if "bf16x2" in insts else None)):
                    if popn is None:
                        continue
                    blocks = np.array_split(np.arange(P), ex_threads)
                    parts = list(ex.map(lambda ix: O.fitness(C_o, popn[ix], want_mag=True), blocks))
                    f_o = np.concatenate([a for a, _ in parts])
                    mag = np.concatenate([b for _, b in parts])
                    f_g = pga.fitness(C, torch.from_numpy(popn).to(dev), "bf16x2", hi=hi, lo=lo).cpu().numpy()
                    d = np.abs(f_g - f_o)
                    rel = d / np.maximum(np.abs(f_o), 1e-300)
                    lg, _, _ = O.best(f_g, popn)
                    lo_, _, _ = O.best(f_o, popn)
                    out[tag] = {"max_rel_err": float(rel.max()), "median_rel_err": float(np.median(rel)),
                                "max_err_over_M": float((d / np.maximum(mag, 1e-300)).max()),
                                "identical_best_labeling": bool(np.array_equal(lg, lo_)),
                                "individuals": int(P)}
            out["note"] = ("every individual's BF16x2 L_c (MFMA pair-sum) against the FP64 oracle's; "
                           "rel = |dL| / |L_oracle|, M = sum of |log terms|")
            return out

        cb = cpu_baseline(w, P, w.seed, gpu_check=gpu_check if "bf16x2" in insts else None)
        pga.route_set(route_default)
        line["cpu_baseline"] = {kk: cb[kk] for kk in ("value", "unit", "cores", "kind", "sample")}
        line["cpu_baseline"]["cpu"] = cb["cpu"]
        if "gpu_vs_oracle" in cb:
            line["precision"]["bf16x2_vs_fp64_oracle"] = cb["gpu_vs_oracle"]
    else:
        line["cpu_baseline"] = None
    ctx.close()
    print(json.dumps(line))


if __name__ == "__main__":
    main()
