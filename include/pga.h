/*
 * pga.h -- C ABI of libpga, the gfx950 (MI355X) library for the master-slave
 * parallel genetic algorithm that maximises the Giada-Marsili cluster
 * likelihood (Hendricks, Gebbie & Wilcox, arXiv 1403.4099).
 *
 * Problem statement followed (Section 2.2.3; Section 4.2.1; Section 5.2.2):
 * the input is the Pearson correlation matrix C of N stocks (Eq. 7); the
 * output is a cluster configuration, one integer label per stock, with the
 * number of clusters left free (labels range over N values, Eq. 9). Fitness
 * is the likelihood L_c of Eq. 8 built from n_s (Eq. 5) and c_s (Eq. 6).
 * The GA follows Algorithm 1 (Section 4.2.3) with every step on the GPU.
 *
 * Conventions for every entry point:
 *   - Array arguments are DEVICE pointers owned by the caller unless marked
 *     "host". The library keeps no pointer after the call returns, except
 *     that work enqueued on `stream` reads and writes them until it runs.
 *   - Matrices are row-major and 0-based. Labels are int32 in [0, N).
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls are asynchronous on that stream unless marked SYNC.
 *   - Return value: PGA_OK, or a negative PGA_ERR_* code detected on the
 *     host from the arguments alone, in which case nothing was enqueued.
 *   - `status` (nullable) is int32[PGA_STATUS_WORDS] on the device. Kernels
 *     add counts to it with integer atomics; the caller zeroes it and reads
 *     it after synchronising the stream. Words:
 *       [PGA_ST_LABEL]     individuals holding a label outside [0, N)
 *       [PGA_ST_DOMAIN]    clusters with n_s > 1 and c_s outside (0, n_s^2)
 *       [PGA_ST_ZEROVAR]   stocks with zero variance (correlation)
 *       [PGA_ST_NONFINITE] individuals whose fitness was set to -inf
 *     An individual counted in LABEL or DOMAIN gets fitness -inf, so it
 *     ranks last and never wins a tournament against a valid one.
 *   - Workspace: entry points that need scratch device memory take
 *     (ws, ws_bytes); the matching *_ws_bytes() function gives the size.
 *     The library allocates no device memory in any of these calls.
 */
#ifndef PGA_H
#define PGA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PGA_OK 0
#define PGA_ERR_ARG (-1)          /* invalid argument (null pointer, size, form, parameter) */
#define PGA_ERR_WORKSPACE (-2)    /* ws null or smaller than the *_ws_bytes() figure */
#define PGA_ERR_HIP (-3)          /* a HIP runtime call failed; see pga_last_hip_error() */
#define PGA_ERR_UNSUPPORTED (-4)  /* size beyond a documented limit (e.g. N > PGA_N_MAX) */

#define PGA_FORM_FP64 0           /* c_s by FP64 masked pair sums on the vector ALUs */
#define PGA_FORM_BF16X2 1         /* c_s by BF16 hi+lo one-hot contraction on MFMA, FP32 accumulate */

#define PGA_STATUS_WORDS 8
#define PGA_ST_LABEL 0
#define PGA_ST_DOMAIN 1
#define PGA_ST_ZEROVAR 2
#define PGA_ST_NONFINITE 3

#define PGA_N_MAX 4096            /* largest number of stocks per instance */
#define PGA_E_MAX 64              /* largest elite count */

#define PGA_SELECT_TOURNAMENT 0   /* parents: winners of tournaments of two */
#define PGA_SELECT_SUS 1          /* parents: stochastic universal sampling after rank scaling */

#define PGA_EWMA_RESET 1          /* pga_ewma: start from a zero covariance state */
#define PGA_EWMA_MARKET 2         /* pga_ewma: remove the equal-weight market return first */

#define PGA_EVOLVE_INIT 1         /* fill pop with the initial population at gen0 first */
#define PGA_EVOLVE_EAGER 2        /* launch kernels one by one instead of replaying a HIP graph */

/* Opaque per-thread context: holds captured HIP graphs and a pinned staging
 * buffer for instance descriptors. Not thread-safe; one per host thread. */
typedef struct pga_ctx pga_ctx;

/* GA parameters of one instance (Table 3 of Section 5.2.1 lists the paper's
 * own; the library uses tournament selection of size 2, uniform crossover and
 * per-gene random-replacement mutation). */
typedef struct {
    int32_t elites;        /* E, 0 <= E < P, E <= PGA_E_MAX (elitism, Section 3.1) */
    int32_t tournament;    /* tournament size; must be 2 with PGA_SELECT_TOURNAMENT */
    uint32_t p_cross_thr;  /* crossover when a uniform u32 is below this (0.9 -> 3865470566) */
    uint32_t p_mut_thr;    /* per-gene mutation when a uniform u32 is below this (1/N -> floor(2^32/N)) */
    uint64_t seed;         /* Philox4x32-10 key: (seed & 0xffffffff, seed >> 32) */
    uint32_t instance_id;  /* goes into every Philox counter; < 2^28 */
    uint32_t gen0;         /* absolute generation index of the population in `pop` on entry */
    int32_t stall_gens;    /* termination test: stop after this many generations without an
                              improvement (Table 3: 50); 0 disables the test */
    int32_t selection;     /* PGA_SELECT_TOURNAMENT or PGA_SELECT_SUS */
    double tol;            /* termination test: an improvement must exceed tol * max(1, |ref|)
                              (Table 3 "error tolerance": 1e-5) */
} pga_params;

/* Termination state of one instance (Algorithm 1, "determine if termination
 * criteria are met"). Device memory owned by the caller; PGA_EVOLVE_INIT
 * resets it, otherwise a call continues from it. After each evaluated
 * generation with best fitness b: b improves on ref when ref is not finite
 * and b is, or when b > ref + tol * max(1, |ref|); an improvement sets
 * ref = b and stall = 0, anything else adds 1 to stall; the instance stops
 * when stall reaches stall_gens. Each generation is tested once: the first
 * evaluation of a call that continues a state which has already tested a
 * generation (ref finite or stall > 0) re-evaluates the population the
 * previous call tested last and leaves the state unchanged, so a run split
 * into several calls equals one call. A stopped instance keeps its population:
 * no later generation of this or any later call evaluates, records
 * statistics rows or breeds it. */
typedef struct {
    double ref;            /* reference best fitness (-inf before the first evaluation) */
    int32_t stall;         /* evaluated generations since the last improvement */
    int32_t stopped;       /* 1 once the test has fired */
    int32_t gens;          /* generations bred, summed over calls (the next call's gen0) */
    int32_t call_gens;     /* generations bred by the latest pga_evolve call */
} pga_term_state;

/* One GA instance. Host struct holding device pointers. */
typedef struct {
    int32_t N;             /* stocks, 1 <= N <= PGA_N_MAX */
    int32_t P;             /* population size, P >= 2 */
    const double *C;       /* N x N correlation, symmetric; the kernels read the diagonal and i < j */
    const uint16_t *C_hi;  /* bf16 hi part, pga_split_ld(N)^2 layout; PGA_FORM_BF16X2 only */
    const uint16_t *C_lo;  /* bf16 lo part, same layout */
    int32_t *pop;          /* P x N labels: generation gen0 on entry, gen0 + G on return */
    int32_t *pop_tmp;      /* P x N scratch, ping-pong partner of pop */
    double *fitness;       /* P: on return, the fitness of the final population */
    double *stats;         /* nullable; (G + 1) x 4 rows {best, mean of finite, #-inf, argbest};
                              rows after a stop are left untouched */
    pga_term_state *term;  /* device; required when prm.stall_gens > 0, else nullable */
    pga_params prm;
} pga_instance;

/* ---- context and errors ------------------------------------------------ */
int pga_ctx_create(pga_ctx **out);
int pga_ctx_destroy(pga_ctx *ctx);
/* Number of captured graphs the context holds (at most 32; the least recently
 * launched is dropped to make room). PGA_ERR_ARG for a null context. */
int pga_ctx_graphs(pga_ctx *ctx);
const char *pga_strerror(int code);
int pga_last_hip_error(void);     /* hipError_t of the last PGA_ERR_HIP on this thread */

/* ---- correlation (Eq. 7) ---------------------------------------------- */
/* C_ij = sum_t x_it x_jt / sqrt(s_i s_j) with x_it = R_it - mean_t R_it and
 * s_i = sum_t x_it^2 (zero-mean data as in Eq. 2; the norm in Eq. 7 is the
 * sum of squares). R: N x T FP64, row stride ld_r >= T. C: N x N FP64 out.
 * C_ii = 1 exactly; off-diagonal values are clamped to [-1, 1]; a stock with
 * s_i = 0 gets 0 off the diagonal and is counted in status[PGA_ST_ZEROVAR].
 * C_hi / C_lo (nullable, both or neither): also write the BF16 split of C
 * (as pga_split). Requires 1 <= N <= PGA_N_MAX, T >= 2. */
/* Workspace: 2N doubles (row means, sums of squares) and the partial Gram
 * tiles of the FP64 MFMA Gram (the t range of each 64 x 64 tile of the upper
 * triangle is split into up to 8 slices, added in slice order). 0 for N < 1
 * or N > PGA_N_MAX. */
size_t pga_correlate_ws_bytes(int32_t N);
int pga_correlate(const double *R, int32_t N, int32_t T, int64_t ld_r, double *C,
                  uint16_t *C_hi, uint16_t *C_lo, int32_t *status, void *ws, size_t ws_bytes,
                  void *stream);

/* ---- BF16 hi + lo split of C (mixed-precision form) ------------------- */
/* Leading dimension (and row count) of the split arrays: N rounded up to 32.
 * Entries outside the N x N corner are written as zero. */
int32_t pga_split_ld(int32_t N);
/* C_hi = bf16(C), C_lo = bf16(C - C_hi), each rounded to nearest, ties to
 * even, from the FP64 value (C - C_hi is exact in FP64). Arrays are
 * pga_split_ld(N) x pga_split_ld(N) uint16 bit patterns. */
int pga_split(const double *C, int32_t N, uint16_t *C_hi, uint16_t *C_lo, void *stream);

/* ---- online EWMA correlation (Section 4.2.5, data pre-processing) ------ */
/* The step before the path for streaming windows: the paper removes the
 * market mode, keeps an exponentially weighted moving-average covariance
 * with forgetting factor lambda (0.98 there), and takes the correlation of
 * that covariance. R: N x T FP64 (row stride ld_r >= T), the T newest
 * returns in time order. S: N x N FP64 covariance state, caller-owned,
 * updated in place (PGA_EWMA_RESET: start from 0; otherwise continue). For
 * each t: m_t = (1/N) sum_i R_it with PGA_EWMA_MARKET, else 0;
 * x_t = R_t - m_t; S <- lambda S + (1 - lambda) x_t x_t^T. Then
 * C_ij = S_ij / sqrt(S_ii S_jj) clamped to [-1, 1], C_ii = 1, and a stock
 * with S_ii = 0 gets 0 off the diagonal and is counted in
 * status[PGA_ST_ZEROVAR]. C_hi / C_lo (nullable, both or neither): also the
 * BF16 split of C as pga_split. Computed as S <- lambda^T S + X X^T with
 * x_it scaled by sqrt((1 - lambda) lambda^(T-1-t)) (FP64 throughout).
 * Errors: PGA_ERR_ARG (null pointer, N < 1, T < 1, ld_r < T, lambda outside
 * [0, 1), unknown flag, one of hi/lo), PGA_ERR_UNSUPPORTED (N > PGA_N_MAX),
 * PGA_ERR_WORKSPACE (pga_ewma_ws_bytes(N, T): the weighted returns, N x T
 * doubles, and the partial Gram tiles as pga_correlate). Async. */
size_t pga_ewma_ws_bytes(int32_t N, int32_t T);
int pga_ewma(const double *R, int32_t N, int32_t T, int32_t ld_r, double lambda, int32_t flags,
             double *S, double *C, uint16_t *C_hi, uint16_t *C_lo, int32_t *status, void *ws,
             size_t ws_bytes, void *stream);

/* ---- fitness (Eqs. 5, 6, 8) -------------------------------------------- */
/* For each of the P labelings (labels: P x N int32):
 *   n_s = #{i : s_i = s}, c_s = sum_{i,j} C_ij [s_i = s][s_j = s] (diagonal
 *   included, computed as sum_i C_ii + 2 sum_{i<j} for symmetric C),
 *   fitness = 1/2 sum_{s: n_s > 1} [log(n_s/c_s) + (n_s-1) log((n_s^2-n_s)/(n_s^2-c_s))]
 * in natural log, literal also when c_s < n_s. n_s (P x N int32) and c_s
 * (P x N FP64), nullable, receive the per-label values (index = label); for
 * an individual with an out-of-range label both rows are zero.
 * form PGA_FORM_FP64: FP64 throughout. form PGA_FORM_BF16X2: the pair sums
 * use C_hi + C_lo on MFMA with FP32 accumulation (flushed to FP64 every 512
 * stocks); diagonal, c_s, logs and the sum over clusters stay FP64.
 * C_hi/C_lo may be NULL for PGA_FORM_FP64. P = 0 is a no-op.
 * Route (both forms, also inside pga_evolve): c_s only involves the pairs
 * within each cluster, so an individual whose clusters hold at most
 * floor(frac * N (N - 1) / 2) pairs (frac: pga_route_get; every pair when
 * N <= 64) and N <= 2048 is evaluated from those pairs alone: FP64 entries of C (diagonal and i < j)
 * summed exactly in 64-bit fixed point, in either form. An individual with a
 * larger pair count, or whose cluster pairs meet an entry with |C_ij| > 1 or
 * not finite, takes the O(N^2) pair-sum of the form as described above. */
size_t pga_fitness_ws_bytes(int32_t N, int32_t P, int32_t form);
int pga_fitness(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
                const int32_t *labels, int32_t P, int32_t form, double *fitness,
                int32_t *n_s, double *c_s, int32_t *status, void *ws, size_t ws_bytes,
                void *stream);

/* ---- fitness without allocation --------------------------------------------
 * For callers that cannot allocate device memory or pass a workspace: code
 * under HIP graph capture, tight serving loops, hosts that forbid hipMalloc.
 * Same computation, arguments and results as pga_fitness, without (ws,
 * ws_bytes): the scratch memory comes from a static device array of
 * PGA_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs
 * on until the process ends (its address is looked up once per device, on
 * the first call with that device current). The call makes no hipMalloc or
 * hipFree and creates no events (kernel timing does not apply to it).
 * Limit: pga_fitness_ws_bytes(N, P, form) <= PGA_NOALLOC_SCRATCH_BYTES, else
 * PGA_ERR_UNSUPPORTED with nothing enqueued (N = 1024, P = 4096 fits in both
 * forms). Every call on one GPU shares that GPU's array, and the array keeps
 * the last call's contents (each call writes all it reads): calls that can
 * overlap on one GPU (different streams, different host threads) race and
 * must be serialised by the caller. Errors otherwise as pga_fitness. Async. */
#define PGA_NOALLOC_SCRATCH_BYTES ((size_t)40 << 20)
size_t pga_fitness_noalloc_max_bytes(void);
int pga_fitness_noalloc(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
                        const int32_t *labels, int32_t P, int32_t form, double *fitness,
                        int32_t *n_s, double *c_s, int32_t *status, void *stream);

/* Cluster-pair route limit (process-wide, read at each call; pga_evolve's
 * cached graphs are keyed by it): frac in [0, 1]; 0 sends every individual to
 * the pair-sum kernels; 1 sends every individual with N <= 2048 to the
 * cluster-pair kernel; any frac > 0 sends every individual with N <= 64 there.
 * PGA_ERR_ARG outside [0, 1] or NaN. */
#define PGA_ROUTE_FRAC_DEFAULT (1.0 / 64.0)
int pga_route_set(double frac);
double pga_route_get(void);

/* ---- kernel variants and autotuning ------------------------------------- */
/* The pair-sum kernel of each form comes in variants that differ only in how
 * work is grouped: individuals per group (per wave for PGA_FORM_FP64, per
 * workgroup for PGA_FORM_BF16X2) and the tile order (xcd_order 0: as
 * launched, column pairs fastest; 1: tiles renumbered so each of the 8 XCDs
 * receives a contiguous range, column pairs fastest; 2: contiguous ranges
 * per XCD with individual batches fastest, so each XCD reads few column
 * blocks of C). All variants of a form
 * give bitwise identical results. pga_fitness and pga_evolve use the variant
 * the process-wide tuning table holds for (form, ceil(N / 64), ceil(log2 P))
 * (N: largest N of the call, P: its total number of individuals), variant 0
 * when there is none; a variant whose LDS does not fit N is replaced by the
 * first variant, in index order, that fits. The table is shared by all
 * threads and devices of the process and guarded by a lock.
 *
 * For PGA_FORM_BF16X2 the variants differ also in their kind:
 *   kind 2 (the default kernel): one column per stock; the one-hot B operand
 *     is read from LDS: an 8-bit row mask per (individual, label code, group
 *     of 8 rows), set by LDS atomics when the rows are staged, indexes a
 *     256-entry table of bf16 one-hot octets;
 *   kind 0: one column per stock, the one-hot built in registers;
 *   kind 1 (packed): columns only for the labels with n_s >= 2 of each
 *     individual's 16-stock tiles, packed over the workgroup's individuals
 *     into groups of 16 (fewer MFMAs, more LDS and scalar work; a small extra
 *     launch marks the labels with n_s >= 2).
 * pga_variant_count: number of variants of `form` (PGA_ERR_ARG for a bad form).
 * pga_variant_info: individuals per group, XCD ordering and kind (each out
 *   pointer nullable) of one variant.
 * pga_tune (SYNC): times every variant that fits N on `labels` (P x N, device):
 *   after 2 reps + 2 warm-up evaluations, three rounds in which each variant
 *   in turn runs `reps` evaluations, all back to back on `stream` and timed
 *   by HIP events (the GPU's clock rises under load, so no variant gains from
 *   its place in the order); stores the fastest in the table (the lowest
 *   variant index among those within 3% of the fastest, the run-to-run spread) and returns it in
 *   out_variant; out_ms (nullable, pga_variant_count(form) floats, host)
 *   receives each variant's best round in milliseconds per evaluation, -1 for
 *   variants that do not fit.
 *   Workspace: pga_tune_ws_bytes(N, P, form). Errors as pga_fitness.
 * pga_tune_set: sets (variant >= 0) or clears (-1) the table entry.
 * pga_tune_get: the variant a call with this (form, N, P) would use. */
int pga_variant_count(int32_t form);
int pga_variant_info(int32_t form, int32_t variant, int32_t *individuals_per_group,
                     int32_t *xcd_order, int32_t *kind);
size_t pga_tune_ws_bytes(int32_t N, int32_t P, int32_t form);
int pga_tune(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
             const int32_t *labels, int32_t P, int32_t form, int32_t reps, void *ws,
             size_t ws_bytes, int32_t *out_variant, float *out_ms, void *stream);
int pga_tune_set(int32_t form, int32_t N, int32_t P, int32_t variant);
int pga_tune_get(int32_t form, int32_t N, int32_t P);
/* Persisted tuning table (host files, SYNC). pga_tune_save writes every entry
 * as a text line "form ceil(N/64) ceil(log2 P) variant" and returns the number
 * of entries; pga_tune_load adds the entries of such a file to the table (an
 * entry replaces the one with the same key) and returns their number. A file
 * that cannot be opened, or a load file with any malformed or out-of-range
 * line (it is then not applied at all): PGA_ERR_ARG. */
int pga_tune_save(const char *path);
int pga_tune_load(const char *path);

/* ---- evolution (Algorithm 1) ------------------------------------------- */
/* Runs `generations` (G >= 0) generations on each of the n_inst instances
 * (inst is a HOST array; the descriptors are copied before return, the
 * buffers they point to are used asynchronously). Per generation g (absolute
 * index gen0 + k): fitness of pop_g; statistics row k; the E fittest copied
 * unchanged to slots 0..E-1 (ties: lower index first); each child slot
 * c >= E gets parents A and B from two tournaments of two (higher fitness
 * wins, ties to the lower index) or, with PGA_SELECT_SUS, by stochastic
 * universal sampling (Section 3.1) after rank scaling: rank r (fitness desc,
 * index asc) weighs floor(sqrt(floor(2^48 / r))), -inf weighs 0 (all 1 if
 * every fitness is -inf); n = 2(P - E) pointers floor((u + k W) / n), W the
 * total weight and u = floor(w W / 2^32) for word 0 w of draw
 * (0, 0xFFFFFFFF, g, SUS), select from the index-ordered segments, and
 * child E + j takes the pointers pi(2j), pi(2j + 1) of a four-round Feistel
 * permutation pi of [0, n) (h-bit halves, 4^h >= n, round function word 0
 * of draw (right half, round, g, SHUFFLE), repeated while >= n); then
 * uniform crossover with probability p_cross and per-gene mutation to a
 * uniform label. After G generations
 * the final population is evaluated into `fitness` and stats row G.
 * Launch sizes are rounded up to one of four values per octave and the
 * instance list padded with empty slots, so a captured graph is replayed for
 * every later call whose instance count, totals of tiles and individuals,
 * largest N and largest P round to the same values (and with the same
 * workspace, status buffer, form, G, kernel variant and route limit); the
 * instances' descriptors are uploaded at each call.
 * Random draws come from Philox4x32-10 with counter
 *   (block, individual or child, generation, tag | instance_id << 4),
 * tags INIT=0, SELECT=1, CROSSOVER=2, MUTATION=3, SUS=4, SHUFFLE=5, so a run is a pure
 * function of (pop at gen0, seed, instance_id, gen0, G): evolving 0->g then
 * g->G equals 0->G bit for bit, alone or batched with other instances.
 * With prm.stall_gens > 0 the termination test (pga_term_state) runs after
 * every evaluation; an instance that stops ends with its last evaluated
 * population in `pop` and its fitness in `fitness`, while the others of the
 * batch go on. flags: PGA_EVOLVE_INIT fills pop at gen0 first (and resets
 * the termination state); PGA_EVOLVE_EAGER skips the HIP graph. All
 * instances use the same `form`. */
size_t pga_evolve_ws_bytes(const pga_instance *inst, int32_t n_inst, int32_t form);
int pga_evolve(pga_ctx *ctx, const pga_instance *inst, int32_t n_inst, int32_t generations,
               int32_t form, int32_t flags, void *ws, size_t ws_bytes, int32_t *status,
               void *stream);

/* ---- result (Algorithm 1 "report on results"; Section 4.2.6) ----------- */
/* SYNC. Picks the fittest of P labelings (lowest index among ties), relabels
 * it in first-occurrence order (first stock's cluster -> 0, next new cluster
 * -> 1, ...; out-of-range labels are copied unchanged), and copies to HOST
 * memory: out_labels (N int32), out_fitness, out_index (each nullable). */
size_t pga_best_ws_bytes(int32_t N);
int pga_best(const double *fitness, const int32_t *labels, int32_t P, int32_t N,
             int32_t *out_labels, double *out_fitness, int32_t *out_index, void *ws,
             size_t ws_bytes, void *stream);

/* ---- kernel timing (measurement support) -------------------------------- */
/* When enabled, every launch of a timed kernel is bracketed by HIP events on
 * the stream it runs on (graph replay is then replaced by eager launches).
 * pga_timing_read synchronises the recorded events and returns the summed
 * elapsed milliseconds and launch count for kernel id
 *   0 pair-sum FP64, 1 pair-sum BF16x2 MFMA, 2 finish (n_s, c_s, L_c),
 *   3 rank/stats, 4 breed, 5 correlate, 6 split, 7 init, 8 SUS ranks and
 *   weights, 9 EWMA correlation, 10 cluster-pair fitness, 11 the labels with
 *   n_s >= 2 (BF16x2 form, before its pair-sum). */
int pga_timing_enable(int on);
int pga_timing_reset(void);
int pga_timing_read(int kernel_id, double *total_ms, int64_t *count);

/* Measurement aid (not part of the method): sustained bf16 MFMA throughput.
 * Launches n_workgroups x 256 threads; every wave issues iters rounds of 16
 * independent v_mfma_f32_16x16x32_bf16 on register operands and writes one
 * float per wave to out (device, caller-owned, 4 * n_workgroups floats; the
 * values only keep the work from being removed). *flops (host, may be NULL)
 * receives the issued flops, n_workgroups * 4 * iters * 16 * 16384; the caller
 * times the launch with events on `stream`. PGA_ERR_ARG for out == NULL,
 * n_workgroups < 1 or iters < 1. Async. */
int pga_peak_mfma_bf16(float *out, int32_t n_workgroups, int32_t iters, double *flops, void *stream);

/* Measurement aid (not part of the method): sustained FP64 vector FMA
 * throughput. Launches n_workgroups x 256 threads; every lane runs iters
 * rounds of 8 independent v_fma_f64 chains on register operands and each wave
 * writes one double to out (device, caller-owned, 4 * n_workgroups doubles).
 * *flops (host, may be NULL) receives n_workgroups * 256 * iters * 8 * 2; the
 * caller times the launch. PGA_ERR_ARG for out == NULL, n_workgroups < 1 or
 * iters < 1. Async. */
int pga_peak_fp64(double *out, int32_t n_workgroups, int32_t iters, double *flops, void *stream);

/* Measurement aid (not part of the method): which pipes of a SIMD overlap.
 * Launches n_workgroups x 256 threads; every wave runs iters rounds of the
 * work `mode` selects (bits): 1 = 4 independent v_mfma_f32_16x16x32_bf16;
 * 2 = the register one-hot of one individual's B operand (4 DPP-broadcast xors
 * and 4 saturating 16-bit subtracts); 4 = 2 ds_read_b128 of conflict-free
 * addresses (with bit 1 they feed the MFMAs); 8 = split: even waves do the
 * MFMA work, odd waves the rest. Accepted modes: 1, 2, 3, 4, 5, 11, 13. Each
 * wave writes one float to out (device, caller-owned, 4 * n_workgroups
 * floats). The caller times the launch with events on `stream` and compares
 * a combined mode's time with its parts' times. PGA_ERR_ARG for out == NULL,
 * another mode, n_workgroups < 1 or iters < 1. Async. */
int pga_pipe_mix(float *out, int32_t mode, int32_t n_workgroups, int32_t iters, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PGA_H */
