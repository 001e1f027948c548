// Host runtime of libpga: the C ABI declared in include/pga.h.
//
// Responsibilities: argument checks (errors are returned before anything is
// enqueued), workspace carving, descriptor upload, the generation schedule
// of Algorithm 1 (fitness -> rank/statistics -> breed, repeated, then a
// final fitness), its capture into a HIP graph that is replayed on later
// calls with the same shapes, the pair-sum kernel variants and their tuning
// table, and optional per-kernel event timing.
#include "pga_internal.hpp"

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <cmath>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

using namespace pga;

// ---- pair-sum kernel variants ----------------------------------------------------
namespace pga {
namespace {
// In order of preference: the tuner gives near-ties (within kTuneTie) to the lower index,
// and variant 0 is the default. XCD order 1 (column pairs fastest) comes first because it
// keeps an individual batch's row labels in the XCD's L2 (a third of the HBM reads of the
// other orders at N = 1024); then order 2, then round-robin tiles.
const Variant kFp64Variants[] = {{PGA_FORM_FP64, 8, 1, 0},  {PGA_FORM_FP64, 16, 1, 0}, {PGA_FORM_FP64, 8, 2, 0},
                                 {PGA_FORM_FP64, 16, 2, 0}, {PGA_FORM_FP64, 8, 0, 0},  {PGA_FORM_FP64, 16, 0, 0}};
// MFMA kernels: the register one-hot column kernel first (the fastest at the
// shapes measured here), then the LDS-table column kernel, then the packed
// (compacted-column) kernel.
const Variant kMfmaVariants[] = {
    {PGA_FORM_BF16X2, 8, 1, kKindCols}, {PGA_FORM_BF16X2, 4, 1, kKindCols},   {PGA_FORM_BF16X2, 16, 1, kKindCols},
    {PGA_FORM_BF16X2, 8, 2, kKindCols}, {PGA_FORM_BF16X2, 4, 2, kKindCols},   {PGA_FORM_BF16X2, 8, 0, kKindCols},
    {PGA_FORM_BF16X2, 4, 1, kKindLut},  {PGA_FORM_BF16X2, 8, 1, kKindLut},    {PGA_FORM_BF16X2, 4, 2, kKindLut},
    {PGA_FORM_BF16X2, 8, 1, kKindPacked}, {PGA_FORM_BF16X2, 16, 1, kKindPacked}, {PGA_FORM_BF16X2, 4, 1, kKindPacked}};
}  // namespace
constexpr int kMaxVariants = 16;
static_assert(sizeof(kMfmaVariants) / sizeof(Variant) <= kMaxVariants &&
                  sizeof(kFp64Variants) / sizeof(Variant) <= kMaxVariants,
              "tuner arrays hold every variant");

int n_variants(int form) {
    if (form == PGA_FORM_FP64) return (int)(sizeof(kFp64Variants) / sizeof(Variant));
    if (form == PGA_FORM_BF16X2) return (int)(sizeof(kMfmaVariants) / sizeof(Variant));
    return 0;
}

Variant variant_at(int form, int idx) {
    return form == PGA_FORM_FP64 ? kFp64Variants[idx] : kMfmaVariants[idx];
}
}  // namespace pga

namespace {

thread_local int g_last_hip = 0;

#define HIP_TRY(expr)                                 \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) {                       \
            g_last_hip = (int)e_;                     \
            return PGA_ERR_HIP;                       \
        }                                             \
    } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// ---- kernel timing -----------------------------------------------------------
struct TimedLaunch {
    int id;
    hipEvent_t a, b;
};
std::mutex g_tmu;
bool g_timing = false;
std::vector<TimedLaunch> g_tl;
constexpr int kTimers = 12;
double g_tsum[kTimers] = {0};
int64_t g_tcnt[kTimers] = {0};

// Set while the allocation-free entry point runs: its launches are never
// bracketed by events (event creation is an allocation).
thread_local bool t_untimed = false;

template <class F>
hipError_t timed(int id, hipStream_t s, F &&launch) {
    if (t_untimed) return launch();
    bool on;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        on = g_timing;
    }
    if (!on) return launch();
    hipEvent_t a, b;
    hipError_t e = hipEventCreate(&a);
    if (e != hipSuccess) return e;
    e = hipEventCreate(&b);
    if (e != hipSuccess) return e;
    e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(g_tmu);
    g_tl.push_back(TimedLaunch{id, a, b});
    return hipSuccess;
}

bool timing_on() {
    std::lock_guard<std::mutex> lk(g_tmu);
    return g_timing;
}

// ---- route limit -----------------------------------------------------------------
// An individual whose clusters hold at most frac * N (N - 1) / 2 pairs is
// evaluated by the cluster-pair kernel; 0 turns that route off. Read at every
// call (and part of a captured graph's key).
std::mutex g_route_mu;
double g_route_frac = PGA_ROUTE_FRAC_DEFAULT;

double route_frac() {
    std::lock_guard<std::mutex> lk(g_route_mu);
    return g_route_frac;
}

// ---- tuning table ----------------------------------------------------------------
// Variant index per (form, ceil(N / 64), ceil(log2 P)); N is the largest N of
// a launch and P its total number of individuals. Filled by pga_tune or
// pga_tune_set; absent keys use variant 0, and a variant whose LDS does not fit
// N is replaced by the first one that does.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tune;

std::tuple<int, int, int> tune_key(int form, int N, int P) {
    int pb = 0;
    while (pb < 31 && (1 << pb) < P) ++pb;
    return std::make_tuple(form, (N + 63) / 64, pb);
}

int pick_variant(int form, int max_n, int total_p) {
    int v = 0;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        auto it = g_tune.find(tune_key(form, max_n, total_p));
        if (it != g_tune.end()) v = it->second;
    }
    if (v >= 0 && v < n_variants(form) && variant_ok(variant_at(form, v), max_n)) return v;
    for (v = 0; v < n_variants(form); ++v)                   // the first variant whose LDS fits max_n
        if (variant_ok(variant_at(form, v), max_n)) return v;
    return 0;
}

// ---- launch sizes of pga_evolve ------------------------------------------------------
// Counts and totals are rounded up to one of four values per octave (x -> the next
// multiple of 2^(floor(log2 x) - 2)), and the instance list is padded with empty
// descriptors (P = 0) to the rounded count: every kernel reads the real totals from
// the device-side prefix tables and skips the workgroups past them, so a captured
// graph serves every mix of instances whose sizes round to the same values (the
// admissions and retirements of a serving loop), with at most a quarter of a launch
// as padding.
int bucket(int x) {
    if (x <= 4) return x;
    int e = 0;
    while ((x >> (e + 1)) != 0) ++e;             // floor(log2 x)
    const int u = 1 << (e - 2);
    return (x + u - 1) / u * u;
}

// ---- workspace layout ----------------------------------------------------------
// [InstDesc x n][prefix tiles n+1][prefix inds n+1][route list counters kListCounters int32]
// [route list entries: list_words(ceil(bucket(sum of P) / 4)) int32]
// then per instance: [wsum P x N doubles][elite PGA_E_MAX int32]
// and, for the BF16x2 form, [hi * 2^125 ld x ld][lo * 2^125 ld x ld] (bf16),
// and, for SUS selection, [rank P int32][weight prefix P uint64],
// then [route P int32][diagonal N + 1 doubles],
// and, for the BF16x2 form, [labels with n_s >= 2: P x ceil(N / 32) uint32].
// Everything a kernel argument points to (the head and the list) sits at an
// offset that depends on n alone, so a captured graph serves every mix of n
// slots; the per-instance regions are reached through the descriptors.
struct Layout {
    size_t desc_off, pre_off, inst_off, list_off;
    std::vector<size_t> wsum_off, elite_off, hs_off, ls_off, rank_off, cum_off, route_off, diag_off, ns2_off;
    size_t total;
};

Layout make_layout(const int32_t *Ns, const int32_t *Ps, int n, int form, const int32_t *sel = nullptr) {
    Layout L;
    L.desc_off = 0;
    L.pre_off = align_up(sizeof(InstDesc) * (size_t)n, 256);
    L.inst_off = align_up(L.pre_off + sizeof(int32_t) * (2 * ((size_t)n + 1) + (size_t)kListCounters), 256);
    L.list_off = L.inst_off;
    int sum_p = 0;
    for (int k = 0; k < n; ++k) sum_p += Ps[k];
    size_t off = align_up(L.list_off + sizeof(int32_t) * list_words((bucket(sum_p) + 3) / 4), 256);
    for (int k = 0; k < n; ++k) {
        L.wsum_off.push_back(off);
        off = align_up(off + sizeof(double) * (size_t)Ns[k] * (size_t)Ps[k], 256);
        L.elite_off.push_back(off);
        off = align_up(off + sizeof(int32_t) * PGA_E_MAX, 256);
        const size_t ld = (size_t)split_ld(Ns[k]);
        const size_t split_bytes = form == PGA_FORM_BF16X2 ? sizeof(uint16_t) * ld * ld : 0;
        L.hs_off.push_back(off);
        off = align_up(off + split_bytes, 256);
        L.ls_off.push_back(off);
        off = align_up(off + split_bytes, 256);
        const bool sus = sel && sel[k] == PGA_SELECT_SUS;
        L.rank_off.push_back(off);
        off = align_up(off + (sus ? sizeof(int32_t) * (size_t)Ps[k] : 0), 256);
        L.cum_off.push_back(off);
        off = align_up(off + (sus ? sizeof(uint64_t) * (size_t)Ps[k] : 0), 256);
        L.route_off.push_back(off);
        off = align_up(off + sizeof(int32_t) * (size_t)Ps[k], 256);
        L.diag_off.push_back(off);
        off = align_up(off + sizeof(double) * ((size_t)Ns[k] + 1), 256);
        L.ns2_off.push_back(off);
        off = align_up(off + (form == PGA_FORM_BF16X2 ? sizeof(uint32_t) * (size_t)Ps[k] * (((size_t)Ns[k] + 31) / 32)
                                                      : 0), 256);
    }
    L.total = off;
    return L;
}

Tables tables_at(void *ws, const Layout &L, int n) {
    char *b = (char *)ws;
    Tables t;
    t.desc = (const InstDesc *)(b + L.desc_off);
    t.tiles = (const int32_t *)(b + L.pre_off);
    t.inds = t.tiles + (n + 1);
    t.sq = (int32_t *)(b + L.pre_off) + 2 * (n + 1);
    t.sq_list = (int32_t *)(b + L.list_off);
    t.n_inst = n;
    return t;
}

// ---- the schedule ----------------------------------------------------------------
struct Shape {
    int n_inst, tiles, inds, max_n;
    Variant v;
    int max_p, sus;      // largest P; 1 if an instance selects by SUS
    int stop;            // 1 if an instance may stop early (termination test on)
    double frac;         // cluster-pair route limit (0: off; then every route pointer is null)
};

// lists_ready: the breed launch that made this population already filled its route lists.
hipError_t run_fitness(const Tables &t, const Shape &sh, int form, int parity, int32_t *status, hipStream_t s,
                       int lists_ready = 0) {
    hipError_t e;
    const int listed = sh.frac > 0.0 && sh.inds >= kManyInds ? 1 : 0;
    if (sh.frac > 0.0 && (e = timed(10, s, [&] {
                              return launch_sparse(t, sh.inds, sh.max_n, parity, sh.frac, listed, lists_ready, status,
                                                   s);
                          })) != hipSuccess)
        return e;
    if (form == PGA_FORM_FP64) {
        e = timed(0, s, [&] { return launch_pairsum_fp64(t, sh.tiles, parity, sh.v, s); });
    } else {
        if (sh.v.kind == kKindPacked &&
            (e = timed(11, s, [&] { return launch_nsmask(t, sh.inds, sh.max_n, parity, s); })) != hipSuccess)
            return e;
        e = timed(1, s, [&] { return launch_pairsum_mfma(t, sh.tiles, parity, sh.v, sh.max_n, s); });
    }
    if (e != hipSuccess) return e;
    return timed(2, s, [&] { return launch_finish(t, sh.inds, sh.max_n, parity, listed, status, s); });
}

hipError_t run_generations(const Tables &t, const Shape &sh, int form, int G, int32_t *status,
                           hipStream_t s) {
    hipError_t e;
    int lists_ready = 0;
    for (int k = 0; k < G; ++k) {
        const int parity = k & 1;
        if ((e = run_fitness(t, sh, form, parity, status, s, lists_ready)) != hipSuccess) return e;
        // Without SUS or an early stop, breeding needs the ranking only for the elite
        // slots, and the breed kernel does it itself (fold); otherwise rank first.
        const int by_wave = sh.max_n <= kBreedWaveMaxN && sh.inds >= kManyInds ? 1 : 0;
        const int fold = (!sh.sus && !sh.stop) ? 1 : 0;
        // with the route lists in use and every N <= 64 (every individual on the cluster-pair
        // route), the wave-per-slot breed fills the next evaluation's list itself
        const int classify = by_wave && sh.frac > 0.0 && sh.max_n <= kRouteAllPairsMaxN ? 1 : 0;
        if (!fold && (e = timed(3, s, [&] { return launch_rank(t, k, 0, s); })) != hipSuccess) return e;
        if (sh.sus && (e = timed(8, s, [&] { return launch_sus(t, sh.max_p, s); })) != hipSuccess) return e;
        if ((e = timed(4, s, [&] {
                 return launch_breed(t, sh.inds, parity, k, fold, by_wave, sh.max_n, classify, s);
             })) != hipSuccess)
            return e;
        lists_ready = classify;
    }
    const int parity = G & 1;
    if ((e = run_fitness(t, sh, form, parity, status, s, lists_ready)) != hipSuccess) return e;
    if ((e = timed(3, s, [&] { return launch_rank(t, G, 1, s); })) != hipSuccess) return e;
    return launch_copy_back(t, sh.inds, G, s);
}

}  // namespace

// ---- context ---------------------------------------------------------------------
struct GraphKey {
    void *ws;
    int32_t *status;
    int n_inst, form, G, tiles, inds, max_n, ipg, order, kind, max_p, sus, stop;
    double frac;
    bool operator<(const GraphKey &o) const {
        return std::tie(ws, status, n_inst, form, G, tiles, inds, max_n, ipg, order, kind, max_p, sus, stop, frac) <
               std::tie(o.ws, o.status, o.n_inst, o.form, o.G, o.tiles, o.inds, o.max_n, o.ipg, o.order, o.kind,
                        o.max_p, o.sus, o.stop, o.frac);
    }
};

struct CachedGraph {
    hipGraph_t graph;
    hipGraphExec_t exec;
    uint64_t last_use;
};
constexpr int kMaxGraphs = 32;                       // captured graphs kept per context (least recently used go)

struct pga_ctx {
    hipStream_t cap = nullptr;
    void *staging = nullptr;
    size_t staging_bytes = 0;
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    uint64_t launches = 0;
    std::map<GraphKey, CachedGraph> graphs;
};

// Measured-ceiling kernel (k_peaks.hip), outside the method's kernels.
namespace pga {
hipError_t launch_peak_mfma(float *out, int n_workgroups, int iters, hipStream_t s);
double peak_mfma_flops(int n_workgroups, int iters);
hipError_t launch_peak_fp64(double *out, int n_workgroups, int iters, hipStream_t s);
double peak_fp64_flops(int n_workgroups, int iters);
hipError_t launch_pipe_mix(float *out, int mode, int n_workgroups, int iters, hipStream_t s);
}  // namespace pga

extern "C" {

int pga_ctx_create(pga_ctx **out) {
    if (!out) return PGA_ERR_ARG;
    pga_ctx *c = new pga_ctx();
    hipError_t e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->upload_done, hipEventDisableTiming);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        delete c;
        return PGA_ERR_HIP;
    }
    *out = c;
    return PGA_OK;
}

int pga_ctx_destroy(pga_ctx *c) {
    if (!c) return PGA_ERR_ARG;
    for (auto &kv : c->graphs) {
        hipGraphExecDestroy(kv.second.exec);
        hipGraphDestroy(kv.second.graph);
    }
    if (c->upload_pending) hipEventSynchronize(c->upload_done);
    if (c->staging) hipHostFree(c->staging);
    if (c->upload_done) hipEventDestroy(c->upload_done);
    if (c->cap) hipStreamDestroy(c->cap);
    delete c;
    return PGA_OK;
}

int pga_ctx_graphs(pga_ctx *c) {
    if (!c) return PGA_ERR_ARG;
    return (int)c->graphs.size();
}

const char *pga_strerror(int code) {
    switch (code) {
        case PGA_OK: return "ok";
        case PGA_ERR_ARG: return "invalid argument";
        case PGA_ERR_WORKSPACE: return "workspace missing or too small";
        case PGA_ERR_HIP: return "HIP runtime error";
        case PGA_ERR_UNSUPPORTED: return "size beyond a documented limit";
        default: return "unknown error";
    }
}

int pga_last_hip_error(void) { return g_last_hip; }
}  // extern "C"

void pga::note_hip_error(int e) { g_last_hip = e; }

extern "C" {

// ---- correlation and split ----------------------------------------------------------
int32_t pga_split_ld(int32_t N) { return N < 1 ? 0 : split_ld(N); }

size_t pga_correlate_ws_bytes(int32_t N) {
    if (N < 1 || N > PGA_N_MAX) return 0;
    return align_up(sizeof(double) * 2 * (size_t)N, 256) + sizeof(double) * gram_ws_doubles(N);
}

int pga_correlate(const double *R, int32_t N, int32_t T, int64_t ld_r, double *C, uint16_t *C_hi,
                  uint16_t *C_lo, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
    if (!R || !C || N < 1 || T < 2 || ld_r < T) return PGA_ERR_ARG;
    if ((C_hi == nullptr) != (C_lo == nullptr)) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pga_correlate_ws_bytes(N)) return PGA_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double *mu = (double *)ws, *ss = mu + N;
    double *part = (double *)((char *)ws + align_up(sizeof(double) * 2 * (size_t)N, 256));
    HIP_TRY(timed(5, s, [&] {
        hipError_t e = launch_row_stats(R, N, T, ld_r, mu, ss, status, s);
        if (e != hipSuccess) return e;
        return launch_corr(R, N, T, ld_r, mu, ss, C, part, s);
    }));
    if (C_hi) HIP_TRY(timed(6, s, [&] { return launch_split(C, N, C_hi, C_lo, s); }));
    return PGA_OK;
}

int pga_split(const double *C, int32_t N, uint16_t *C_hi, uint16_t *C_lo, void *stream) {
    if (!C || !C_hi || !C_lo || N < 1) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(timed(6, s, [&] { return launch_split(C, N, C_hi, C_lo, s); }));
    return PGA_OK;
}

// ---- online EWMA correlation -------------------------------------------------------------
size_t pga_ewma_ws_bytes(int32_t N, int32_t T) {
    if (N < 1 || T < 1 || N > PGA_N_MAX) return 0;
    return align_up(sizeof(double) * (size_t)N * (size_t)T, 256) + sizeof(double) * gram_ws_doubles(N);
}

int pga_ewma(const double *R, int32_t N, int32_t T, int32_t ld_r, double lambda, int32_t flags, double *S,
             double *C, uint16_t *C_hi, uint16_t *C_lo, int32_t *status, void *ws, size_t ws_bytes,
             void *stream) {
    if (!R || !S || !C || N < 1 || T < 1 || ld_r < T) return PGA_ERR_ARG;
    if (!(lambda >= 0.0 && lambda < 1.0)) return PGA_ERR_ARG;
    if ((C_hi == nullptr) != (C_lo == nullptr)) return PGA_ERR_ARG;
    if (flags & ~(PGA_EWMA_RESET | PGA_EWMA_MARKET)) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    if (!ws || ws_bytes < pga_ewma_ws_bytes(N, T)) return PGA_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    double *part = (double *)((char *)ws + align_up(sizeof(double) * (size_t)N * (size_t)T, 256));
    HIP_TRY(timed(9, s, [&] {
        return launch_ewma(R, N, T, ld_r, lambda, (flags & PGA_EWMA_RESET) ? 1 : 0,
                           (flags & PGA_EWMA_MARKET) ? 1 : 0, S, C, (double *)ws, part, status, s);
    }));
    if (C_hi) HIP_TRY(timed(6, s, [&] { return launch_split(C, N, C_hi, C_lo, s); }));
    return PGA_OK;
}

// ---- fitness -----------------------------------------------------------------------------
size_t pga_fitness_ws_bytes(int32_t N, int32_t P, int32_t form) {
    if (N < 1 || P < 0) return 0;
    const Layout L = make_layout(&N, &P, 1, form);
    return L.total;
}

namespace {
// Checks, descriptor and (BF16x2) scaled split for a single-instance fitness
// launch; run_fitness then evaluates labels into `fitness`.
int prepare_single(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
                   const int32_t *labels, int32_t P, int32_t form, double *fitness, int32_t *n_s,
                   double *c_s, void *ws, size_t ws_bytes, hipStream_t s, Tables *t, Shape *sh,
                   InstDesc *dd, double frac) {
    if (N < 1 || P < 0) return PGA_ERR_ARG;
    if (form != PGA_FORM_FP64 && form != PGA_FORM_BF16X2) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    if (P == 0) return PGA_OK;
    if (!C || !labels || !fitness) return PGA_ERR_ARG;
    if (form == PGA_FORM_BF16X2 && (!C_hi || !C_lo)) return PGA_ERR_ARG;
    const Layout L = make_layout(&N, &P, 1, form);
    if (!ws || ws_bytes < L.total) return PGA_ERR_WORKSPACE;

    InstDesc d{};
    d.N = N;
    d.P = P;
    d.E = 0;
    d.ld_h = split_ld(N);
    d.C = C;
    d.hi = C_hi;
    d.lo = C_lo;
    d.pop[0] = const_cast<int32_t *>(labels);
    d.pop[1] = nullptr;
    d.fitness = fitness;
    d.wsum = (double *)((char *)ws + L.wsum_off[0]);
    d.elite = (int32_t *)((char *)ws + L.elite_off[0]);
    if (form == PGA_FORM_BF16X2) {
        d.hs = (uint16_t *)((char *)ws + L.hs_off[0]);
        d.ls = (uint16_t *)((char *)ws + L.ls_off[0]);
        d.ns2 = (uint32_t *)((char *)ws + L.ns2_off[0]);
    }
    d.n_s_out = n_s;
    d.c_s_out = c_s;
    if (frac > 0.0) {
        d.route = (int32_t *)((char *)ws + L.route_off[0]);
        d.diag = (double *)((char *)ws + L.diag_off[0]);
    }
    *t = tables_at(ws, L, 1);
    sh->n_inst = 1;
    sh->inds = P;
    sh->max_n = N;
    sh->max_p = P;
    sh->sus = 0;
    sh->stop = 0;
    sh->frac = frac;
    *dd = d;
    if (form == PGA_FORM_BF16X2) {
        HIP_TRY(launch_write_desc(d, 0, (InstDesc *)t->desc, (int32_t *)t->tiles, s));
        HIP_TRY(launch_scale_split(*t, d.ld_h, s));
    }
    return PGA_OK;
}

// Writes the tile prefix of variant v into the descriptor area and sets sh.
hipError_t use_variant(const InstDesc &d, const Tables &t, int form, int vi, Shape *sh, hipStream_t s) {
    sh->v = variant_at(form, vi);
    sh->tiles = pair_tiles(d.N, d.P, sh->v);
    return launch_write_desc(d, sh->tiles, (InstDesc *)t.desc, (int32_t *)t.tiles, s);
}
}  // namespace

int pga_fitness(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
                const int32_t *labels, int32_t P, int32_t form, double *fitness, int32_t *n_s,
                double *c_s, int32_t *status, void *ws, size_t ws_bytes, void *stream) {
    return pga::fitness_call(C, C_hi, C_lo, N, labels, P, form, fitness, n_s, c_s, status, ws, ws_bytes,
                             (hipStream_t)stream, true);
}
}  // extern "C"

namespace pga {
int fitness_call(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N, const int32_t *labels,
                 int32_t P, int32_t form, double *fitness, int32_t *n_s, double *c_s, int32_t *status, void *ws,
                 size_t ws_bytes, hipStream_t s, bool timing_allowed) {
    struct Untimed {
        bool prev;
        explicit Untimed(bool on) : prev(t_untimed) { t_untimed = prev || on; }
        ~Untimed() { t_untimed = prev; }
    } guard(!timing_allowed);
    Tables t;
    Shape sh;
    InstDesc d;
    const int rc = prepare_single(C, C_hi, C_lo, N, labels, P, form, fitness, n_s, c_s, ws, ws_bytes, s,
                                  &t, &sh, &d, route_frac());
    if (rc != PGA_OK || P == 0) return rc;
    HIP_TRY(use_variant(d, t, form, pick_variant(form, N, P), &sh, s));
    if (sh.frac > 0.0) HIP_TRY(launch_diag(t, N, s));
    HIP_TRY(run_fitness(t, sh, form, 0, status, s));
    return PGA_OK;
}
}  // namespace pga

extern "C" {

// ---- autotuning ---------------------------------------------------------------------------
int pga_variant_count(int32_t form) {
    const int n = n_variants(form);
    return n > 0 ? n : PGA_ERR_ARG;
}

int pga_variant_info(int32_t form, int32_t variant, int32_t *ipg, int32_t *xcd_order, int32_t *kind) {
    if (variant < 0 || variant >= n_variants(form)) return PGA_ERR_ARG;
    const Variant v = variant_at(form, variant);
    if (ipg) *ipg = v.ipg;
    if (xcd_order) *xcd_order = v.order;
    if (kind) *kind = v.kind;
    return PGA_OK;
}

int pga_tune_get(int32_t form, int32_t N, int32_t P) {
    if (n_variants(form) == 0 || N < 1 || P < 1) return PGA_ERR_ARG;
    return pick_variant(form, N, P);
}

int pga_tune_set(int32_t form, int32_t N, int32_t P, int32_t variant) {
    if (n_variants(form) == 0 || N < 1 || P < 1 || variant < -1 || variant >= n_variants(form))
        return PGA_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (variant < 0) g_tune.erase(tune_key(form, N, P));
    else g_tune[tune_key(form, N, P)] = variant;
    return PGA_OK;
}

// Tuning table file: one line per entry, "form n64 log2p variant" (n64 = ceil(N / 64),
// log2p = ceil(log2 P), the table's own key), '#' starts a comment line.
int pga_tune_save(const char *path) {
    if (!path) return PGA_ERR_ARG;
    std::map<std::tuple<int, int, int>, int> copy;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        copy = g_tune;
    }
    FILE *f = fopen(path, "w");
    if (!f) return PGA_ERR_ARG;
    fprintf(f, "# libpga pair-sum variants: form ceil(N/64) ceil(log2 P) variant\n");
    for (const auto &kv : copy)
        fprintf(f, "%d %d %d %d\n", std::get<0>(kv.first), std::get<1>(kv.first), std::get<2>(kv.first), kv.second);
    const int bad = ferror(f);
    if (fclose(f) != 0 || bad) return PGA_ERR_ARG;
    return (int)copy.size();
}

int pga_tune_load(const char *path) {
    if (!path) return PGA_ERR_ARG;
    FILE *f = fopen(path, "r");
    if (!f) return PGA_ERR_ARG;
    std::map<std::tuple<int, int, int>, int> read;
    char line[256];
    int rc = PGA_OK;
    while (fgets(line, sizeof line, f)) {
        if (line[0] == '#' || line[0] == '\n') continue;
        int form, nb, pb, v;
        if (sscanf(line, "%d %d %d %d", &form, &nb, &pb, &v) != 4 || n_variants(form) == 0 || nb < 1 ||
            nb > (PGA_N_MAX + 63) / 64 || pb < 0 || pb > 31 || v < 0 || v >= n_variants(form)) {
            rc = PGA_ERR_ARG;                         // the whole file is rejected
            break;
        }
        read[std::make_tuple(form, nb, pb)] = v;
    }
    fclose(f);
    if (rc != PGA_OK) return rc;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto &kv : read) g_tune[kv.first] = kv.second;
    return (int)read.size();
}

size_t pga_tune_ws_bytes(int32_t N, int32_t P, int32_t form) {
    const size_t base = pga_fitness_ws_bytes(N, P, form);
    if (base == 0) return 0;
    return base + align_up(sizeof(double) * (size_t)P, 256) + align_up(sizeof(int32_t) * PGA_STATUS_WORDS, 256);
}

int pga_tune(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
             const int32_t *labels, int32_t P, int32_t form, int32_t reps, void *ws, size_t ws_bytes,
             int32_t *out_variant, float *out_ms, void *stream) {
    if (reps < 1 || P < 1) return PGA_ERR_ARG;
    const size_t need = pga_tune_ws_bytes(N, P, form);
    if (need == 0) return N > PGA_N_MAX ? PGA_ERR_UNSUPPORTED : PGA_ERR_ARG;
    if (!ws || ws_bytes < need) return PGA_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    const size_t base = pga_fitness_ws_bytes(N, P, form);
    double *fit = (double *)((char *)ws + base);
    int32_t *st = (int32_t *)((char *)ws + base + align_up(sizeof(double) * (size_t)P, 256));
    Tables t;
    Shape sh;
    InstDesc d;
    // The variants differ only in the pair-sum kernel, so every individual takes that route here.
    int rc = prepare_single(C, C_hi, C_lo, N, labels, P, form, fit, nullptr, nullptr, ws, base, s, &t, &sh, &d,
                            0.0);
    if (rc != PGA_OK) return rc;
    // The GPU's clock rises under sustained load, so the variants are timed round-robin over
    // kTuneRounds rounds after a warm-up, back to back with no host synchronisation between
    // them, and each keeps its fastest round: no variant is favoured by its place in the order.
    constexpr int kTuneRounds = 3;
    constexpr float kTuneTie = 0.03f;
    int valid[kMaxVariants];
    int nvalid = 0;
    for (int vi = 0; vi < n_variants(form); ++vi) {
        if (variant_ok(variant_at(form, vi), N)) valid[nvalid++] = vi;
        else if (out_ms) out_ms[vi] = -1.f;
    }
    if (nvalid == 0) return PGA_ERR_UNSUPPORTED;
    const int nseg = kTuneRounds * nvalid;
    hipEvent_t ev[2 * kTuneRounds * kMaxVariants] = {};
    hipError_t e = hipSuccess;
    int created = 0;
    for (; created < 2 * nseg && e == hipSuccess; ++created) e = hipEventCreate(&ev[created]);
    if (e != hipSuccess) --created;
    if (e == hipSuccess) e = use_variant(d, t, form, valid[0], &sh, s);
    for (int r = 0; r < 2 * reps + 2 && e == hipSuccess; ++r) e = run_fitness(t, sh, form, 0, st, s);   // warm-up
    for (int seg = 0; seg < nseg && e == hipSuccess; ++seg) {
        if ((e = use_variant(d, t, form, valid[seg % nvalid], &sh, s)) != hipSuccess) break;
        if ((e = hipEventRecord(ev[2 * seg], s)) != hipSuccess) break;
        for (int r = 0; r < reps && e == hipSuccess; ++r) e = run_fitness(t, sh, form, 0, st, s);
        if (e == hipSuccess) e = hipEventRecord(ev[2 * seg + 1], s);
    }
    if (e == hipSuccess) e = hipEventSynchronize(ev[2 * nseg - 1]);
    float seg_ms[kMaxVariants];
    for (int k = 0; k < nvalid; ++k) seg_ms[k] = -1.f;
    for (int seg = 0; seg < nseg && e == hipSuccess; ++seg) {
        float ms = 0.f;
        if ((e = hipEventElapsedTime(&ms, ev[2 * seg], ev[2 * seg + 1])) != hipSuccess) break;
        ms /= (float)reps;
        float &m = seg_ms[seg % nvalid];
        if (m < 0.f || ms < m) m = ms;
    }
    for (int i = 0; i < created; ++i) hipEventDestroy(ev[i]);
    if (e != hipSuccess) {
        g_last_hip = (int)e;
        return PGA_ERR_HIP;
    }
    float best_ms = -1.f;
    for (int k = 0; k < nvalid; ++k) {
        if (out_ms) out_ms[valid[k]] = seg_ms[k];
        if (best_ms < 0.f || seg_ms[k] < best_ms) best_ms = seg_ms[k];
    }
    int best = valid[0];
    for (int k = nvalid - 1; k >= 0; --k)                 // lowest index within kTuneTie of the fastest
        if (seg_ms[k] <= best_ms * (1.f + kTuneTie)) best = valid[k];
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        g_tune[tune_key(form, N, P)] = best;
    }
    if (out_variant) *out_variant = best;
    return PGA_OK;
}

// ---- evolution ----------------------------------------------------------------------------
static int check_instances(const pga_instance *inst, int32_t n, int32_t form) {
    if (!inst || n < 1) return PGA_ERR_ARG;
    for (int k = 0; k < n; ++k) {
        const pga_instance &I = inst[k];
        if (I.N < 1 || I.P < 2) return PGA_ERR_ARG;
        if (I.N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
        if (!I.C || !I.pop || !I.pop_tmp || !I.fitness) return PGA_ERR_ARG;
        if (form == PGA_FORM_BF16X2 && (!I.C_hi || !I.C_lo)) return PGA_ERR_ARG;
        if (I.prm.elites < 0 || I.prm.elites >= I.P || I.prm.elites > PGA_E_MAX) return PGA_ERR_ARG;
        if (I.prm.selection != PGA_SELECT_TOURNAMENT && I.prm.selection != PGA_SELECT_SUS) return PGA_ERR_ARG;
        if (I.prm.selection == PGA_SELECT_TOURNAMENT && I.prm.tournament != 2) return PGA_ERR_ARG;
        if (I.prm.instance_id >= (1u << 28)) return PGA_ERR_ARG;
        if (I.prm.stall_gens < 0 || std::isnan(I.prm.tol)) return PGA_ERR_ARG;
        if (I.prm.stall_gens > 0 && !I.term) return PGA_ERR_ARG;
    }
    return PGA_OK;
}

size_t pga_evolve_ws_bytes(const pga_instance *inst, int32_t n_inst, int32_t form) {
    if (check_instances(inst, n_inst, form) != PGA_OK) return 0;
    const int nb = bucket(n_inst);
    std::vector<int32_t> Ns(nb, 0), Ps(nb, 0), Ss(nb, 0);
    for (int k = 0; k < n_inst; ++k) {
        Ns[k] = inst[k].N;
        Ps[k] = inst[k].P;
        Ss[k] = inst[k].prm.selection;
    }
    return make_layout(Ns.data(), Ps.data(), nb, form, Ss.data()).total;
}

int pga_evolve(pga_ctx *ctx, const pga_instance *inst, int32_t n_inst, int32_t generations,
               int32_t form, int32_t flags, void *ws, size_t ws_bytes, int32_t *status, void *stream) {
    if (!ctx || generations < 0) return PGA_ERR_ARG;
    if (form != PGA_FORM_FP64 && form != PGA_FORM_BF16X2) return PGA_ERR_ARG;
    int rc = check_instances(inst, n_inst, form);
    if (rc != PGA_OK) return rc;
    const int nb = bucket(n_inst);                   // descriptor slots: the instances, then padding
    std::vector<int32_t> Ns(nb, 0), Ps(nb, 0), Ss(nb, 0);
    for (int k = 0; k < n_inst; ++k) {
        Ns[k] = inst[k].N;
        Ps[k] = inst[k].P;
        Ss[k] = inst[k].prm.selection;
    }
    const Layout L = make_layout(Ns.data(), Ps.data(), nb, form, Ss.data());
    if (!ws || ws_bytes < L.total) return PGA_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;

    // host image of the descriptor table and prefix arrays
    const size_t head = L.inst_off;
    if (ctx->upload_pending) {
        HIP_TRY(hipEventSynchronize(ctx->upload_done));
        ctx->upload_pending = false;
    }
    if (ctx->staging_bytes < head) {
        if (ctx->staging) HIP_TRY(hipHostFree(ctx->staging));
        ctx->staging = nullptr;
        ctx->staging_bytes = 0;
        HIP_TRY(hipHostMalloc(&ctx->staging, head, hipHostMallocDefault));
        ctx->staging_bytes = head;
    }
    char *hb = (char *)ctx->staging;
    InstDesc *hd = (InstDesc *)(hb + L.desc_off);
    int32_t *pf = (int32_t *)(hb + L.pre_off);
    int32_t *pi = pf + (nb + 1);
    pf[0] = pi[0] = 0;
    memset(pi + (nb + 1), 0, sizeof(int32_t) * kListCounters);     // the route lists start empty
    Shape sh{nb, 0, 0, 0, Variant{form, 0, 0, 0}, 0, 0, 0, route_frac()};
    int total_p = 0;
    for (int k = 0; k < n_inst; ++k) {
        sh.max_n = std::max(sh.max_n, (int)inst[k].N);
        sh.max_p = std::max(sh.max_p, (int)inst[k].P);
        sh.sus |= inst[k].prm.selection == PGA_SELECT_SUS ? 1 : 0;
        sh.stop |= inst[k].prm.stall_gens > 0 ? 1 : 0;
        total_p += inst[k].P;
    }
    sh.max_n = bucket(sh.max_n);
    sh.max_p = bucket(sh.max_p);
    sh.v = variant_at(form, pick_variant(form, sh.max_n, total_p));
    for (int k = 0; k < n_inst; ++k) {
        const pga_instance &I = inst[k];
        InstDesc d{};
        d.N = I.N;
        d.P = I.P;
        d.E = I.prm.elites;
        d.ld_h = split_ld(I.N);
        d.C = I.C;
        d.hi = I.C_hi;
        d.lo = I.C_lo;
        d.pop[0] = I.pop;
        d.pop[1] = I.pop_tmp;
        d.fitness = I.fitness;
        d.stats = I.stats;
        d.wsum = (double *)((char *)ws + L.wsum_off[k]);
        d.elite = (int32_t *)((char *)ws + L.elite_off[k]);
        if (form == PGA_FORM_BF16X2) {
            d.hs = (uint16_t *)((char *)ws + L.hs_off[k]);
            d.ls = (uint16_t *)((char *)ws + L.ls_off[k]);
            d.ns2 = (uint32_t *)((char *)ws + L.ns2_off[k]);
        }
        d.p_cross = I.prm.p_cross_thr;
        d.p_mut = I.prm.p_mut_thr;
        d.seed = I.prm.seed;
        d.inst_id = I.prm.instance_id;
        d.gen0 = I.prm.gen0;
        d.term = I.term;
        d.stall_gens = I.prm.stall_gens;
        d.tol = I.prm.tol;
        d.selection = I.prm.selection;
        if (I.prm.selection == PGA_SELECT_SUS) {
            d.sus_rank = (int32_t *)((char *)ws + L.rank_off[k]);
            d.sus_cum = (uint64_t *)((char *)ws + L.cum_off[k]);
        }
        if (sh.frac > 0.0) {
            d.route = (int32_t *)((char *)ws + L.route_off[k]);
            d.diag = (double *)((char *)ws + L.diag_off[k]);
        }
        d.ind0 = pi[k];
        hd[k] = d;
        pf[k + 1] = pf[k] + pair_tiles(I.N, I.P, sh.v);
        pi[k + 1] = pi[k] + I.P;
    }
    for (int k = n_inst; k < nb; ++k) {              // padding slots: no individuals, no tiles
        hd[k] = InstDesc{};
        pf[k + 1] = pf[k];
        pi[k + 1] = pi[k];
    }
    sh.tiles = bucket(pf[nb]);                       // launch sizes; the kernels stop at the real totals
    sh.inds = bucket(pi[nb]);
    HIP_TRY(hipMemcpyAsync(ws, ctx->staging, head, hipMemcpyHostToDevice, s));
    HIP_TRY(hipEventRecord(ctx->upload_done, s));
    ctx->upload_pending = true;

    Tables t = tables_at(ws, L, nb);
    if (form == PGA_FORM_BF16X2) HIP_TRY(launch_scale_split(t, split_ld(sh.max_n), s));
    if (sh.frac > 0.0) HIP_TRY(launch_diag(t, sh.max_n, s));
    if (flags & PGA_EVOLVE_INIT) HIP_TRY(timed(7, s, [&] { return launch_init(t, sh.inds, s); }));

    const bool eager = (flags & PGA_EVOLVE_EAGER) || timing_on();
    if (eager) {
        HIP_TRY(run_generations(t, sh, form, generations, status, s));
        return PGA_OK;
    }
    GraphKey key{ws, status, nb, form, generations, sh.tiles, sh.inds, sh.max_n, sh.v.ipg, sh.v.order, sh.v.kind,
                 sh.max_p, sh.sus, sh.stop, sh.frac};
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        // bounded cache: drop the least recently launched graph
        if ((int)ctx->graphs.size() >= kMaxGraphs) {
            auto old = ctx->graphs.begin();
            for (auto g = ctx->graphs.begin(); g != ctx->graphs.end(); ++g)
                if (g->second.last_use < old->second.last_use) old = g;
            hipGraphExecDestroy(old->second.exec);
            hipGraphDestroy(old->second.graph);
            ctx->graphs.erase(old);
        }
        hipGraph_t g = nullptr;
        hipGraphExec_t ge = nullptr;
        HIP_TRY(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
        hipError_t e = run_generations(t, sh, form, generations, status, ctx->cap);
        hipError_t e2 = hipStreamEndCapture(ctx->cap, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            g_last_hip = (int)(e != hipSuccess ? e : e2);
            return PGA_ERR_HIP;
        }
        e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(g);
            g_last_hip = (int)e;
            return PGA_ERR_HIP;
        }
        it = ctx->graphs.emplace(key, CachedGraph{g, ge, 0}).first;
    }
    it->second.last_use = ++ctx->launches;
    HIP_TRY(hipGraphLaunch(it->second.exec, s));
    return PGA_OK;
}

// ---- best ------------------------------------------------------------------------------------
size_t pga_best_ws_bytes(int32_t N) {
    if (N < 1) return 0;
    return align_up(sizeof(int32_t) * ((size_t)N + 1), 256) + 256;
}

int pga_best(const double *fitness, const int32_t *labels, int32_t P, int32_t N, int32_t *out_labels,
             double *out_fitness, int32_t *out_index, void *ws, size_t ws_bytes, void *stream) {
    if (!fitness || !labels || P < 1 || N < 1) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    const size_t need = pga_best_ws_bytes(N);
    if (!ws || ws_bytes < need) return PGA_ERR_WORKSPACE;
    hipStream_t s = (hipStream_t)stream;
    int32_t *dl = (int32_t *)ws;
    double *df = (double *)((char *)ws + align_up(sizeof(int32_t) * ((size_t)N + 1), 256));
    HIP_TRY(launch_best(fitness, labels, P, N, dl, df, s));
    std::vector<int32_t> hl((size_t)N + 1);
    double hf = 0.0;
    HIP_TRY(hipMemcpyAsync(hl.data(), dl, sizeof(int32_t) * ((size_t)N + 1), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hf, df, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (out_labels) for (int i = 0; i < N; ++i) out_labels[i] = hl[i];
    if (out_fitness) *out_fitness = hf;
    if (out_index) *out_index = hl[N];
    return PGA_OK;
}

// ---- route limit ----------------------------------------------------------------------------
int pga_route_set(double frac) {
    if (!(frac >= 0.0 && frac <= 1.0)) return PGA_ERR_ARG;
    std::lock_guard<std::mutex> lk(g_route_mu);
    g_route_frac = frac;
    return PGA_OK;
}

double pga_route_get(void) { return route_frac(); }

// ---- timing ----------------------------------------------------------------------------------
int pga_timing_enable(int on) {
    std::lock_guard<std::mutex> lk(g_tmu);
    g_timing = on != 0;
    return PGA_OK;
}

static int drain_timing() {
    std::vector<TimedLaunch> v;
    {
        std::lock_guard<std::mutex> lk(g_tmu);
        v.swap(g_tl);
    }
    for (auto &x : v) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(x.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, x.a, x.b);
        hipEventDestroy(x.a);
        hipEventDestroy(x.b);
        if (e != hipSuccess) {
            g_last_hip = (int)e;
            return PGA_ERR_HIP;
        }
        std::lock_guard<std::mutex> lk(g_tmu);
        g_tsum[x.id] += ms;
        g_tcnt[x.id] += 1;
    }
    return PGA_OK;
}

int pga_timing_reset(void) {
    int rc = drain_timing();
    std::lock_guard<std::mutex> lk(g_tmu);
    for (int i = 0; i < kTimers; ++i) {
        g_tsum[i] = 0.0;
        g_tcnt[i] = 0;
    }
    return rc;
}

int pga_peak_mfma_bf16(float *out, int32_t n_workgroups, int32_t iters, double *flops, void *stream) {
    if (!out || n_workgroups < 1 || iters < 1) return PGA_ERR_ARG;
    if (flops) *flops = pga::peak_mfma_flops(n_workgroups, iters);
    HIP_TRY(pga::launch_peak_mfma(out, n_workgroups, iters, (hipStream_t)stream));
    return PGA_OK;
}

int pga_peak_fp64(double *out, int32_t n_workgroups, int32_t iters, double *flops, void *stream) {
    if (!out || n_workgroups < 1 || iters < 1) return PGA_ERR_ARG;
    if (flops) *flops = pga::peak_fp64_flops(n_workgroups, iters);
    HIP_TRY(pga::launch_peak_fp64(out, n_workgroups, iters, (hipStream_t)stream));
    return PGA_OK;
}

int pga_pipe_mix(float *out, int32_t mode, int32_t n_workgroups, int32_t iters, void *stream) {
    const bool known = mode == 1 || mode == 2 || mode == 3 || mode == 4 || mode == 5 || mode == 11 || mode == 13;
    if (!out || !known || n_workgroups < 1 || iters < 1) return PGA_ERR_ARG;
    HIP_TRY(pga::launch_pipe_mix(out, mode, n_workgroups, iters, (hipStream_t)stream));
    return PGA_OK;
}

int pga_timing_read(int kernel_id, double *total_ms, int64_t *count) {
    if (kernel_id < 0 || kernel_id >= kTimers) return PGA_ERR_ARG;
    int rc = drain_timing();
    if (rc != PGA_OK) return rc;
    std::lock_guard<std::mutex> lk(g_tmu);
    if (total_ms) *total_ms = g_tsum[kernel_id];
    if (count) *count = g_tcnt[kernel_id];
    return PGA_OK;
}

}  // extern "C"
