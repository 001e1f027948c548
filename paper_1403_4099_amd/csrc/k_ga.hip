// Genetic-algorithm kernels (Algorithm 1 of Section 4.2.3; operators of
// Section 3.1): initial population, ranking and statistics, the fused
// breed step (elitism + tournament selection + uniform crossover +
// mutation + replacement into the other ping-pong buffer), and the
// report of the fittest labeling in canonical form.
//
// Random numbers: Philox4x32-10, counter (block, individual or child,
// generation, tag | instance << 4), key = seed. A draw is keyed by the
// absolute generation and the instance id, never by launch layout, so a run
// gives the same bits alone or inside a batch and across resumes.
#include "pga_internal.hpp"

#include <math.h>

namespace pga {

// ---------------------------------------------------------------------------
// Initial population: gene i of individual p is scale_u32(word i%4 of draw
// (i/4, p, gen0, INIT), N). One workgroup per individual.
__global__ __launch_bounds__(256) void k_init(Tables t) {
    const int g = blockIdx.x;
    if (g >= t.inds[t.n_inst]) return;                     // the grid may exceed the total (capacity-sized graph)
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int N = d.N;
    const int p = g - t.inds[k];
    if (p == 0 && threadIdx.x == 0 && d.term) {
        pga_term_state z;
        z.ref = -INFINITY;
        z.stall = z.stopped = z.gens = z.call_gens = 0;
        *d.term = z;
    }
    int32_t *__restrict__ row = d.pop[0] + (size_t)p * N;
    const int nq = (N + 3) >> 2;
    for (int q = threadIdx.x; q < nq; q += 256) {
        const U4 w = draw((uint32_t)q, (uint32_t)p, d.gen0, kTagInit, d.inst_id, d.seed);
        const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 4 * q + r;
            if (i < N) row[i] = (int32_t)scale_u32(ws[r], (uint32_t)N);
        }
    }
}

hipError_t launch_init(Tables t, int total_inds, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3(total_inds), dim3(256), 0, s, t);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ranking and statistics: one workgroup per instance. Elite r is the best
// individual ranked after elite r-1 in the total order (fitness desc, index
// asc), found by a block arg-best reduction; the order is total, so the
// result does not depend on the reduction's shape. Statistics row gen_off:
// {best, mean of finite fitnesses (-inf if none), #-inf, argbest}.
struct Cand {
    double f;
    int i;
};

__device__ Cand block_best(Cand c, double *rf, int *ri) {
    rf[threadIdx.x] = c.f;
    ri[threadIdx.x] = c.i;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            const double fo = rf[threadIdx.x + w];
            const int io = ri[threadIdx.x + w];
            const int im = ri[threadIdx.x];
            if (io >= 0 && (im < 0 || ranks_before(fo, io, rf[threadIdx.x], im))) {
                rf[threadIdx.x] = fo;
                ri[threadIdx.x] = io;
            }
        }
        __syncthreads();
    }
    Cand r{rf[0], ri[0]};
    __syncthreads();
    return r;
}

// Wave butterflies: the comparison is a total order and the sums run in a fixed
// pattern, so every lane ends with the same, reproducible value.
__device__ __forceinline__ Cand wave_best(Cand c) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const double fo = __shfl_xor(c.f, m, 64);
        const int io = __shfl_xor(c.i, m, 64);
        if (io >= 0 && (c.i < 0 || ranks_before(fo, io, c.f, c.i))) c = Cand{fo, io};
    }
    return c;
}

__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Elite selection, termination state and statistics of one instance by one
// workgroup of kRankThreads threads: the rank kernel, and, when the breed
// kernel does the ranking itself (no SUS, no early stop), the breed workgroups
// of the elite slots. Both use this code with the same thread count, so their
// statistics agree bit for bit. Each thread keeps up to CACHE of its fitness
// values in registers (all loads issued at once) and re-reads the rest; every
// thread visits its values in the same order whatever CACHE is, so CACHE
// changes no result.
constexpr int kRankThreads = 256;
constexpr int kRankWaves = kRankThreads / 64;
constexpr int kRankCache = 16;

struct RankLds {
    double wf[kRankWaves];
    int wi[kRankWaves];
};

template <int CACHE>
struct RankBlock {
    const double *__restrict__ f;
    int P;
    RankLds &sh;
    double fr[CACHE];

    __device__ void load() {
#pragma unroll
        for (int v = 0; v < CACHE; ++v) {
            const int p = threadIdx.x + v * kRankThreads;
            fr[v] = p < P ? gld(f + p) : -INFINITY;
        }
    }
    // Best candidate of this thread ranked after prev (prev.i < 0: no bound).
    __device__ Cand thread_best(Cand prev) const {
        Cand c{0.0, -1};
#pragma unroll
        for (int v = 0; v < CACHE; ++v) {
            const int p = threadIdx.x + v * kRankThreads;
            if (p >= P) break;
            if (prev.i >= 0 && !ranks_before(prev.f, prev.i, fr[v], p)) continue;
            if (c.i < 0 || ranks_before(fr[v], p, c.f, c.i)) c = Cand{fr[v], p};
        }
        for (int p0 = threadIdx.x + CACHE * kRankThreads; p0 < P; p0 += 4 * kRankThreads) {
            double fq[4];                                  // four loads in flight, then the compares
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * kRankThreads;
                fq[u] = p < P ? gld(f + p) : -INFINITY;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * kRankThreads;
                if (p >= P) break;
                if (prev.i >= 0 && !ranks_before(prev.f, prev.i, fq[u], p)) continue;
                if (c.i < 0 || ranks_before(fq[u], p, c.f, c.i)) c = Cand{fq[u], p};
            }
        }
        return c;
    }
    __device__ Cand block_best(Cand c) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        c = wave_best(c);
        if (lane == 0) {
            sh.wf[wave] = c.f;
            sh.wi[wave] = c.i;
        }
        __syncthreads();
        Cand b{0.0, -1};
        for (int w = 0; w < kRankWaves; ++w)
            if (sh.wi[w] >= 0 && (b.i < 0 || ranks_before(sh.wf[w], sh.wi[w], b.f, b.i))) b = Cand{sh.wf[w], sh.wi[w]};
        __syncthreads();
        return b;
    }
    __device__ double block_sum(double v) {
        const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
        v = wave_sum_d(v);
        if (lane == 0) sh.wf[wave] = v;
        __syncthreads();
        double r = 0.0;
        for (int w = 0; w < kRankWaves; ++w) r += sh.wf[w];
        __syncthreads();
        return r;
    }
    // The r-th ranked individual for r = 0 .. rounds-1: calls visit(r, cand) in order.
    template <typename F>
    __device__ void ranked(int rounds, F &&visit) {
        Cand prev{0.0, -1};
        for (int r = 0; r < rounds; ++r) {
            const Cand b = block_best(thread_best(prev));
            visit(r, b);
            prev = b;
        }
    }
    // Ranks 0 .. rounds-1 (rounds <= kTop) from ONE read of the values: each
    // thread keeps its kTop best in rank order, and round r takes the best of the
    // threads' heads (the r-th ranked individual cannot be a thread's (kTop+1)-th
    // best). The same read accumulates the statistics partials in the order
    // write_stats takes them.
    static constexpr int kTop = 4;
    template <typename F>
    __device__ void ranked_once(int rounds, double &sum, double &ninv, F &&visit) {
        Cand top[kTop];
#pragma unroll
        for (int k = 0; k < kTop; ++k) top[k] = Cand{0.0, -1};
        sum = 0.0;
        ninv = 0.0;
        auto take = [&](double fp, int p) {
            if (isfinite(fp)) sum += fp;
            else ninv += 1.0;
            Cand x{fp, p};
#pragma unroll
            for (int k = 0; k < kTop; ++k)
                if (x.i >= 0 && (top[k].i < 0 || ranks_before(x.f, x.i, top[k].f, top[k].i))) {
                    const Cand y = top[k];
                    top[k] = x;
                    x = y;
                }
        };
#pragma unroll
        for (int v = 0; v < CACHE; ++v) {
            const int p = threadIdx.x + v * kRankThreads;
            if (p >= P) break;
            take(fr[v], p);
        }
        for (int p0 = threadIdx.x + CACHE * kRankThreads; p0 < P; p0 += 4 * kRankThreads) {
            double fq[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * kRankThreads;
                fq[u] = p < P ? gld(f + p) : -INFINITY;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int p = p0 + u * kRankThreads;
                if (p >= P) break;
                take(fq[u], p);
            }
        }
        for (int r = 0; r < rounds; ++r) {
            const Cand b = block_best(top[0]);
            if (b.i >= 0 && b.i == top[0].i) {                 // this thread's head was taken
#pragma unroll
                for (int k = 0; k + 1 < kTop; ++k) top[k] = top[k + 1];
                top[kTop - 1] = Cand{0.0, -1};
            }
            visit(r, b);
        }
    }
    // Ranks 0 .. rounds-1 (visit(r, cand) in order) and, with stats set, the
    // statistics row gen_off; returns the best. A single read of the values
    // serves up to kTop ranks, more take one read per rank.
    template <typename F>
    __device__ Cand rank_and_stats(const InstDesc &d, int rounds, int gen_off, bool stats, F &&visit) {
        Cand best{-INFINITY, 0};
        if (rounds <= kTop) {
            double sum, ninv;
            ranked_once(rounds, sum, ninv, [&](int r, Cand b) {
                if (r == 0) best = b;
                visit(r, b);
            });
            if (stats) store_stats(d, gen_off, best, block_sum(sum), block_sum(ninv));
        } else {
            ranked(rounds, [&](int r, Cand b) {
                if (r == 0) best = b;
                visit(r, b);
            });
            if (stats) write_stats(d, gen_off, best);
        }
        return best;
    }
    // Statistics row gen_off: {best, mean of finite fitnesses (-inf if none), #-inf, argbest}.
    __device__ void write_stats(const InstDesc &d, int gen_off, Cand best) {
        double sum = 0.0, ninv = 0.0;
#pragma unroll
        for (int v = 0; v < CACHE; ++v) {
            const int p = threadIdx.x + v * kRankThreads;
            if (p >= P) break;
            if (isfinite(fr[v])) sum += fr[v];
            else ninv += 1.0;
        }
        for (int p = threadIdx.x + CACHE * kRankThreads; p < P; p += kRankThreads) {
            const double fp = gld(f + p);
            if (isfinite(fp)) sum += fp;
            else ninv += 1.0;
        }
        store_stats(d, gen_off, best, block_sum(sum), block_sum(ninv));
    }
    __device__ void store_stats(const InstDesc &d, int gen_off, Cand best, double total, double inv) const {
        if (threadIdx.x == 0) {
            double *row = d.stats + 4 * (size_t)gen_off;
            const double nfin = (double)P - inv;
            row[0] = best.f;
            row[1] = nfin > 0.0 ? total / nfin : -INFINITY;
            row[2] = inv;
            row[3] = (double)best.i;
        }
    }
};

// Termination state after this generation's best b (thread 0 of the ranking
// workgroup): improvement, stall count, stop flag; the generation about to be
// bred is counted unless this is the final evaluation or the run stopped.
// Algorithm 1 tests each generation once: the first evaluation of a call
// (first != 0) re-evaluates the population a previous call tested last when
// the state has already tested a generation (ref finite or stall > 0), and
// then does not enter the test again, so a run split into several calls is
// the same run as one call.
__device__ void term_update(const InstDesc &d, pga_term_state st, double b, int final, int first) {
    const bool retest = first && (isfinite(st.ref) || st.stall != 0);
    if (!retest) {
        const bool improved = isfinite(st.ref) ? (b > st.ref + d.tol * fmax(1.0, fabs(st.ref))) : isfinite(b);
        if (improved) {
            st.ref = b;
            st.stall = 0;
        } else {
            st.stall += 1;
        }
        if (d.stall_gens > 0 && st.stall >= d.stall_gens) st.stopped = 1;
    }
    if (!final && !st.stopped) {
        st.gens += 1;
        st.call_gens += 1;
    }
    *d.term = st;
}

__global__ __launch_bounds__(kRankThreads) void k_rank(Tables t, int gen_off, int final) {
    __shared__ RankLds sh;
    const InstDesc &d = t.desc[blockIdx.x];
    if (d.P == 0) return;                                  // a padding slot of a capacity-sized launch
    const int P = d.P, E = d.E;
    // The fitness values, the stop flag and (thread 0) the termination state are
    // all requested before any of them is used.
    RankBlock<kRankCache> rb{d.fitness, P, sh};
    rb.load();
    pga_term_state st{};
    if (d.term) {
        const bool stopped = inst_stopped(d);
        if (threadIdx.x == 0) st = *d.term;
        __syncthreads();                                   // every thread has read the flag
        if (gen_off == 0 && threadIdx.x == 0) {
            gst(&d.term->call_gens, 0);
            st.call_gens = 0;
        }
        if (stopped) return;
    }
    if (d.selection == PGA_SELECT_SUS)                     // the SUS rank kernel adds into these
        for (int p = threadIdx.x; p < P; p += kRankThreads) gst(d.sus_rank + p, 1);
    const Cand best = rb.rank_and_stats(d, E > 1 ? E : 1, gen_off, d.stats != nullptr, [&](int r, Cand b) {
        if (r < E && threadIdx.x == 0) d.elite[r] = b.i;
    });
    if (d.term && threadIdx.x == 0) term_update(d, st, best.f, final, gen_off == 0);
}

hipError_t launch_rank(Tables t, int gen_off, int final, hipStream_t s) {
    hipLaunchKernelGGL(k_rank, dim3(t.n_inst), dim3(kRankThreads), 0, s, t, gen_off, final);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Breed: one workgroup per slot c of the next population.
//   c < E : copy elite c unchanged (elitism).
//   c >= E: parents A, B = winners of two tournaments of two on draw
//           (0, c, g, SELECT); crossover iff word 0 of (0, c, g, CROSSOVER)
//           < p_cross, and then gene j from B iff bit j%32 of word (j%128)/32
//           of (1 + j/128, c, g, CROSSOVER); mutation of gene j iff word
//           2(j%2) of (j/2, c, g, MUTATION) < p_mut, new label from the
//           next word.
// Each thread takes gene pairs (j, j+1) so one mutation draw covers two
// genes; one wave covers 128 genes, so the crossover-bit draw is the same
// for the whole wave.
__device__ __forceinline__ int tournament2(const double *f, int a, int b) {
    const double fa = f[a], fb = f[b];
    return ranks_before(fa, a, fb, b) ? a : b;
}

// ---------------------------------------------------------------------------
// Stochastic universal sampling after rank scaling (PGA_SELECT_SUS).
//   k_sus_rank:   rank_p = 1 + #{q : q ranks before p}; workgroup (x, y, inst)
//                 compares individuals [256x, 256x + 256) with [256y, 256y + 256)
//                 and adds its integer counts atomically (exact, order-free);
//   k_sus_prefix: weight floor(sqrt(floor(2^48 / rank))) (0 for -inf, 1 for all
//                 when every fitness is -inf) and the inclusive prefix over the
//                 individuals in index order, in 64-bit integers;
//   k_breed:      pointer k at floor((u + k W) / n) picks the individual whose
//                 segment holds it; child E + j uses pointers pi(2j), pi(2j+1).
__global__ __launch_bounds__(256) void k_sus_rank(Tables t) {
    __shared__ double fq[256];
    const InstDesc &d = t.desc[blockIdx.z];
    if (d.P == 0 || d.selection != PGA_SELECT_SUS || inst_stopped(d)) return;
    const int P = d.P;
    const int p0 = blockIdx.x * 256, q0 = blockIdx.y * 256;
    if (p0 >= P || q0 >= P) return;                          // uniform over the workgroup
    const int p = p0 + threadIdx.x, q = q0 + threadIdx.x;
    fq[threadIdx.x] = q < P ? gld(d.fitness + q) : 0.0;
    __syncthreads();
    if (p >= P) return;
    const double fp = gld(d.fitness + p);
    const int nq = min(256, P - q0);
    int cnt = 0;
    for (int r = 0; r < nq; ++r) cnt += ranks_before(fq[r], q0 + r, fp, p) ? 1 : 0;
    if (cnt) atomicAdd(d.sus_rank + p, cnt);
}

__device__ __forceinline__ uint64_t isqrt_u48(uint64_t x) {
    uint64_t y = (uint64_t)sqrt((double)x);                 // within one of the exact root
    while (y * y > x) --y;
    while ((y + 1) * (y + 1) <= x) ++y;
    return y;
}

__global__ __launch_bounds__(1024) void k_sus_prefix(Tables t) {
    __shared__ uint64_t wsum[16];
    __shared__ uint64_t carry_s;
    const InstDesc &d = t.desc[blockIdx.x];
    if (d.P == 0 || d.selection != PGA_SELECT_SUS || inst_stopped(d)) return;
    const int P = d.P;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    for (int pass = 0; pass < 2; ++pass) {                   // pass 1 only if every weight was 0
        uint64_t carry = 0;
        for (int base = 0; base < P; base += 1024) {
            const int p = base + threadIdx.x;
            uint64_t w = 0;
            if (p < P) {
                if (pass == 1) w = 1;
                else if (isfinite(gld(d.fitness + p)))
                    w = isqrt_u48(((uint64_t)1 << 48) / (uint64_t)gld(d.sus_rank + p));
            }
            uint64_t x = w;                                  // inclusive scan over the wave
#pragma unroll
            for (int o = 1; o < 64; o <<= 1) {
                const uint64_t y = __shfl_up(x, o, 64);
                if (lane >= o) x += y;
            }
            if (lane == 63) wsum[wave] = x;
            __syncthreads();
            uint64_t before = carry;
            for (int v = 0; v < wave; ++v) before += wsum[v];
            if (p < P) gst(d.sus_cum + p, before + x);
            if (threadIdx.x == 1023) carry_s = before + x;
            __syncthreads();
            carry = carry_s;
            __syncthreads();
        }
        if (carry != 0) break;
    }
}

hipError_t launch_sus(Tables t, int max_p, hipStream_t s) {
    if (t.n_inst <= 0 || max_p <= 0) return hipSuccess;
    const int nb = (max_p + 255) / 256;
    hipLaunchKernelGGL(k_sus_rank, dim3(nb, nb, t.n_inst), dim3(256), 0, s, t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sus_prefix, dim3(t.n_inst), dim3(1024), 0, s, t);
    return hipGetLastError();
}

// Image of x under the Feistel permutation of [0, n) that pairs SUS parents.
__device__ uint32_t shuffle_index(uint32_t x, uint32_t n, const InstDesc &d, uint32_t gen) {
    int h = 1;
    while (((uint64_t)1 << (2 * h)) < (uint64_t)n) ++h;
    const uint32_t mask = (1u << h) - 1u;
    do {
        uint32_t L = x >> h, R = x & mask;
        for (uint32_t round = 0; round < 4; ++round) {
            const uint32_t t = R;
            R = L ^ (draw(R, round, gen, kTagShuf, d.inst_id, d.seed).x & mask);
            L = t;
        }
        x = (L << h) | R;
    } while (x >= n);
    return x;
}

// Individual whose SUS segment holds pointer k (smallest p with cum[p] > pos).
__device__ int sus_pick(const InstDesc &d, uint32_t k, uint32_t n, uint64_t u, uint64_t W) {
    const uint64_t pos = (u + (uint64_t)k * W) / (uint64_t)n;
    int lo = 0, hi = d.P - 1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (gld(d.sus_cum + mid) > pos) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Parent pair of child c (c >= E): two tournaments of two on draw (0, c, g,
// SELECT), or, with SUS, the individuals under shuffled pointers 2(c - E) and
// 2(c - E) + 1 (which = 0, 1).
__device__ int sus_parent(const InstDesc &d, int c, uint32_t gen, int which) {
    const int P = d.P, E = d.E;
    const uint32_t n = 2u * (uint32_t)(P - E);
    const uint64_t W = gld(d.sus_cum + (P - 1));
    const uint32_t w0 = draw(0u, 0xFFFFFFFFu, gen, kTagSus, d.inst_id, d.seed).x;
    const uint64_t u = __umul64hi((uint64_t)w0 << 32, W);              // floor(w0 W / 2^32)
    const uint32_t k = shuffle_index(2u * (uint32_t)(c - E) + (uint32_t)which, n, d, gen);
    return sus_pick(d, k, n, u, W);
}

// Genes of child c from parents A and B (crossover and mutation), written to
// out by `width` threads with index tid: a whole workgroup or one wave. Every
// draw is keyed by gene pair, so the child does not depend on the split. One
// wave covers 128 consecutive genes per pass in either split, so the
// crossover-bit draw is the same for the whole wave.
__device__ __forceinline__ void breed_genes(const InstDesc &d, int c, uint32_t gen, const int32_t *__restrict__ ra,
                                            const int32_t *__restrict__ rb, int32_t *__restrict__ out, int tid,
                                            int width) {
    const int N = d.N;
    const bool cross = draw(0u, (uint32_t)c, gen, kTagXov, d.inst_id, d.seed).x < d.p_cross;
    const uint32_t pm = d.p_mut;
    const int npair = (N + 1) >> 1;
    for (int jp = tid; jp < npair; jp += width) {
        const int j = 2 * jp;
        const bool has1 = j + 1 < N;
        int32_t g0 = ra[j];
        int32_t g1 = has1 ? ra[j + 1] : 0;
        if (cross) {
            const uint32_t q = __builtin_amdgcn_readfirstlane((uint32_t)(j >> 7));
            const U4 xb = draw(1u + q, (uint32_t)c, gen, kTagXov, d.inst_id, d.seed);
            const int r = j & 127;
            const int wsel = r >> 5;
            const uint32_t word = wsel == 0 ? xb.x : wsel == 1 ? xb.y : wsel == 2 ? xb.z : xb.w;
            const int bit = r & 31;
            if ((word >> bit) & 1u) g0 = rb[j];
            if (has1 && ((word >> (bit + 1)) & 1u)) g1 = rb[j + 1];
        }
        const U4 m = draw((uint32_t)jp, (uint32_t)c, gen, kTagMut, d.inst_id, d.seed);
        if (m.x < pm) g0 = (int32_t)scale_u32(m.y, (uint32_t)N);
        if (m.z < pm) g1 = (int32_t)scale_u32(m.w, (uint32_t)N);
        out[j] = g0;
        if (has1) out[j + 1] = g1;
    }
}

// With `fold` set (no instance selects by SUS or can stop early), the breed
// workgroups of the elite slots rank the population themselves: workgroup
// c < E finds the c-th ranked individual and copies it, and workgroup 0 also
// keeps the termination state and writes the statistics row, so the rank
// kernel is not launched between fitness and breeding. Children need only the
// fitness values (tournaments), so the result is the same as with the rank
// kernel before breed.
__global__ __launch_bounds__(256) void k_breed(Tables t, int parity, int gen_off, int fold) {
    const int g = blockIdx.x;
    if (g >= t.inds[t.n_inst]) return;                     // the grid may exceed the total (capacity-sized graph)
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;                           // set by this generation's rank
    const int N = d.N, P = d.P, E = d.E;
    const int c = g - t.inds[k];
    const int32_t *__restrict__ src = d.pop[parity];
    int32_t *__restrict__ out = d.pop[parity ^ 1] + (size_t)c * N;

    // Ranking work of the fold: workgroup c < E finds the c-th ranked individual;
    // workgroup 0 (an elite slot, or child 0 when E = 0) keeps the termination
    // state and writes the statistics row. The condition is uniform per workgroup.
    int ec = -1;
    if (fold && (c < E || (c == 0 && (d.term || d.stats)))) {
        __shared__ RankLds sh;
        RankBlock<4> rb{d.fitness, P, sh};                    // few registers: the child slots share the kernel
        rb.load();
        pga_term_state st{};
        if (c == 0 && d.term && threadIdx.x == 0) st = *d.term;
        Cand pick{-INFINITY, 0};
        const Cand best = rb.rank_and_stats(d, c + 1, gen_off, c == 0 && d.stats, [&](int, Cand b) { pick = b; });
        if (c == 0 && d.term && threadIdx.x == 0) {
            if (gen_off == 0) st.call_gens = 0;
            term_update(d, st, best.f, 0, gen_off == 0);
        }
        ec = pick.i;
    }
    if (c < E) {
        if (!fold) ec = d.elite[c];
        const int32_t *__restrict__ e = src + (size_t)ec * N;
        for (int j = threadIdx.x; j < N; j += 256) out[j] = e[j];
        return;
    }
    const uint32_t gen = d.gen0 + (uint32_t)gen_off;
    int A, B;
    if (d.selection == PGA_SELECT_SUS) {
        __shared__ int par_s[2];
        if (threadIdx.x < 2) par_s[threadIdx.x] = sus_parent(d, c, gen, threadIdx.x);
        __syncthreads();
        A = par_s[0];
        B = par_s[1];
    } else {
        const double *__restrict__ f = d.fitness;
        const U4 sel = draw(0u, (uint32_t)c, gen, kTagSel, d.inst_id, d.seed);
        A = tournament2(f, (int)scale_u32(sel.x, (uint32_t)P), (int)scale_u32(sel.y, (uint32_t)P));
        B = tournament2(f, (int)scale_u32(sel.z, (uint32_t)P), (int)scale_u32(sel.w, (uint32_t)P));
    }
    breed_genes(d, c, gen, src + (size_t)A * N, src + (size_t)B * N, out, threadIdx.x, 256);
}

// The same step with one wave per slot of the next population (four slots per
// workgroup, possibly of different instances): at small N a workgroup per slot
// leaves most of its threads idle and bounds the slots in flight by the
// workgroup limit per compute unit. With `fold` set, workgroup k < n_inst
// ranks instance k instead (the same RankBlock code and thread count as the
// rank kernel, so the statistics are the same bits), copies its elites and
// keeps its termination state and statistics row, and the slot workgroups
// follow; otherwise the elite slots copy the individuals the rank kernel
// listed.
// classify (every N <= 64): also append the elites to the next evaluation's
// sparse list.
__device__ __forceinline__ void fold_rank(const Tables &t, int k, int parity, int gen_off, int classify, int slices,
                                          int cap) {
    __shared__ RankLds sh;
    const InstDesc &d = t.desc[k];
    const int P = d.P, E = d.E, N = d.N;
    if (P == 0 || (E == 0 && !d.term && !d.stats)) return;   // a padding slot, or nothing to rank
    // This workgroup's chain of reductions is the longest path of the launch:
    // its waves issue ahead of the slot waves that share their SIMDs.
    __builtin_amdgcn_s_setprio(3);
    RankBlock<4> rb{d.fitness, P, sh};                     // the slot waves share the register budget
    rb.load();
    pga_term_state st{};
    if (d.term && threadIdx.x == 0) st = *d.term;
    const int32_t *__restrict__ src = d.pop[parity];
    int32_t *__restrict__ dst = d.pop[parity ^ 1];
    // Up to four elites are copied after the ranking, their loads in flight
    // together; more are copied as they are found.
    constexpr int kQ = RankBlock<4>::kTop;
    int eq[kQ] = {0, 0, 0, 0};
    const Cand best = rb.rank_and_stats(d, E > 1 ? E : 1, gen_off, d.stats != nullptr, [&](int r, Cand b) {
        if (r >= E) return;
        if (E <= kQ) {
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                if (q == r) eq[q] = b.i;
            return;
        }
        const int32_t *__restrict__ e = src + (size_t)b.i * N;
        int32_t *__restrict__ o = dst + (size_t)r * N;
        for (int j = threadIdx.x; j < N; j += kRankThreads) o[j] = e[j];
    });
    if (d.term && threadIdx.x == 0) {
        if (gen_off == 0) st.call_gens = 0;
        term_update(d, st, best.f, 0, gen_off == 0);
    }
    if (E <= kQ)
        for (int j = threadIdx.x; j < N; j += kRankThreads) {
            int32_t v[kQ];
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                if (q < E) v[q] = src[(size_t)eq[q] * N + j];
#pragma unroll
            for (int q = 0; q < kQ; ++q)
                if (q < E) dst[(size_t)q * N + j] = v[q];
        }
    if (classify && threadIdx.x == 0)
        for (int r = 0; r < E; ++r) route_append(t, d, k, r, t.inds[k] + r, parity ^ 1, kListSparse, slices, cap);
}

// The slot workgroups are taken XCD by XCD: the x-th eighth of them runs on XCD
// x (workgroup i goes to XCD i mod 8), so the parents an XCD reads come from a
// few instances' populations and stay in its L2.
// GL lanes per slot: 64 (one wave), or 32 and 16 when the launch's largest N
// is at most 2 GL genes (a lane makes two genes per pass), so that a wave
// breeds 64 / GL children at the paper's sizes (N = 18) instead of keeping 55
// of its 64 lanes idle. The lanes of one slot share its instance and child,
// so their control flow is the same.
// classify (the launch's largest N is at most 64, so every individual takes
// the cluster-pair route): the writer of each slot (the slot's lanes, or the
// ranking workgroup for the elites it copies) appends it to the next
// evaluation's sparse list, and workgroup 0 empties this parity's lists, which
// the evaluation just done used; that evaluation then needs no route kernel.
template <int GL>
__global__ __launch_bounds__(256) void k_breed_wave(Tables t, int parity, int gen_off, int fold, int slot_wgs,
                                                    int classify, int slices, int cap) {
    constexpr int S = 64 / GL;                             // slots per wave
    if (classify && blockIdx.x == 0)
        for (int i = threadIdx.x; i < 2 * kListSlices; i += 256) gst(list_count(t, parity, 0, 0) + i, 0);
    int wg = blockIdx.x;
    if (fold) {
        if (wg < t.n_inst) {
            fold_rank(t, wg, parity, gen_off, classify, slices, cap);
            return;
        }
        wg -= t.n_inst;
    }
    wg = (wg % kXcds) * (slot_wgs / kXcds) + wg / kXcds;  // slot_wgs is a multiple of 8
    const int lane = threadIdx.x & 63, sub = lane / GL, gl = lane % GL;
    int g = (4 * wg + (int)(threadIdx.x >> 6)) * S + sub;
    if constexpr (GL == 64) g = __builtin_amdgcn_readfirstlane(g);
    if (g >= t.inds[t.n_inst]) return;                     // the grid may exceed the total (capacity-sized graph)
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;                           // set by this generation's rank
    const int N = d.N, P = d.P, E = d.E;
    const int c = g - t.inds[k];
    const int32_t *__restrict__ src = d.pop[parity];
    int32_t *__restrict__ out = d.pop[parity ^ 1] + (size_t)c * N;
    auto finish_slot = [&]() {
        if (classify && gl == 0) route_append(t, d, k, c, g, parity ^ 1, kListSparse, slices, cap);
    };
    if (c < E) {
        if (fold) return;                                  // copied by the instance's ranking workgroup
        const int32_t *__restrict__ e = src + (size_t)d.elite[c] * N;
        for (int j = gl; j < N; j += GL) out[j] = e[j];
        finish_slot();
        return;
    }
    const uint32_t gen = d.gen0 + (uint32_t)gen_off;
    int A, B;
    if (d.selection == PGA_SELECT_SUS) {
        int pick = 0;
        if (gl < 2) pick = sus_parent(d, c, gen, gl);
        if constexpr (GL == 64) {
            A = __builtin_amdgcn_readlane(pick, 0);
            B = __builtin_amdgcn_readlane(pick, 1);
        } else {                                           // from the slot's first two lanes
            A = __shfl(pick, sub * GL, 64);
            B = __shfl(pick, sub * GL + 1, 64);
        }
    } else {
        const double *__restrict__ f = d.fitness;
        const U4 sel = draw(0u, (uint32_t)c, gen, kTagSel, d.inst_id, d.seed);
        A = tournament2(f, (int)scale_u32(sel.x, (uint32_t)P), (int)scale_u32(sel.y, (uint32_t)P));
        B = tournament2(f, (int)scale_u32(sel.z, (uint32_t)P), (int)scale_u32(sel.w, (uint32_t)P));
    }
    breed_genes(d, c, gen, src + (size_t)A * N, src + (size_t)B * N, out, gl, GL);
    finish_slot();
}

hipError_t launch_breed(Tables t, int total_inds, int parity, int gen_off, int fold, int by_wave, int max_n,
                        int classify, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    if (by_wave) {
        const int gl = max_n <= 32 ? 16 : max_n <= 64 ? 32 : 64;   // lanes per slot
        const int per_wg = 4 * (64 / gl);                          // slots per workgroup
        const int slot_wgs = ((total_inds + per_wg - 1) / per_wg + kXcds - 1) / kXcds * kXcds;
        const int n_wg = (total_inds + 3) / 4, slices = list_slices(n_wg), cap = list_slice_cap(n_wg);
        const dim3 grid((fold ? t.n_inst : 0) + slot_wgs);
        if (gl == 16)
            hipLaunchKernelGGL(k_breed_wave<16>, grid, dim3(256), 0, s, t, parity, gen_off, fold, slot_wgs, classify,
                               slices, cap);
        else if (gl == 32)
            hipLaunchKernelGGL(k_breed_wave<32>, grid, dim3(256), 0, s, t, parity, gen_off, fold, slot_wgs, classify,
                               slices, cap);
        else
            hipLaunchKernelGGL(k_breed_wave<64>, grid, dim3(256), 0, s, t, parity, gen_off, fold, slot_wgs, classify,
                               slices, cap);
    }
    else
        hipLaunchKernelGGL(k_breed, dim3(total_inds), dim3(256), 0, s, t, parity, gen_off, fold);
    return hipGetLastError();
}

// After an odd number of bred generations the population sits in pop[1]; copy
// it back so the caller always finds the result in the buffer it passed as
// pop. Without a termination test every call breeds G generations.
__global__ __launch_bounds__(256) void k_copy_back(Tables t, int G) {
    const int g = blockIdx.x;
    if (g >= t.inds[t.n_inst]) return;                     // the grid may exceed the total (capacity-sized graph)
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int bred = d.term ? gld(&d.term->call_gens) : G;
    if ((bred & 1) == 0) return;
    const int N = d.N;
    const int p = g - t.inds[k];
    const int32_t *__restrict__ a = d.pop[1] + (size_t)p * N;
    int32_t *__restrict__ b = d.pop[0] + (size_t)p * N;
    for (int j = threadIdx.x; j < N; j += 256) b[j] = a[j];
}

hipError_t launch_copy_back(Tables t, int total_inds, int G, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_back, dim3(total_inds), dim3(256), 0, s, t, G);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Best: arg-best over P (lowest index among ties), then relabel that row in
// first-occurrence order. first[s] = smallest stock index carrying label s
// (integer atomicMin, order-free); stock i opens a new cluster iff
// first[s_i] == i; the new label of s is the number of clusters opened
// before first[s] (exclusive scan). Out-of-range labels are copied through.
// out[0..N) = labels, out[N] = index; out_f = fitness.
__global__ __launch_bounds__(256) void k_best(const double *f, const int32_t *labels, int P, int N,
                                               int32_t *out, double *out_f) {
    __shared__ double rf[256];
    __shared__ int ri[256];
    __shared__ int first[PGA_N_MAX];
    __shared__ int open[PGA_N_MAX];
    __shared__ int part[256];

    Cand c{0.0, -1};
    for (int p = threadIdx.x; p < P; p += 256)
        if (c.i < 0 || ranks_before(f[p], p, c.f, c.i)) c = Cand{f[p], p};
    const Cand b = block_best(c, rf, ri);
    const int32_t *__restrict__ row = labels + (size_t)b.i * N;

    for (int s = threadIdx.x; s < N; s += 256) first[s] = 0x7fffffff;
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += 256) {
        const int l = row[i];
        if (l >= 0 && l < N) atomicMin(&first[l], i);
    }
    __syncthreads();
    // contiguous chunk per thread, then an exclusive scan of chunk totals
    const int chunk = (N + 255) / 256;
    const int i0 = threadIdx.x * chunk, i1 = min(N, i0 + chunk);
    int local = 0;
    for (int i = i0; i < i1; ++i) {
        const int l = row[i];
        const int o = (l >= 0 && l < N && first[l] == i) ? 1 : 0;
        open[i] = local;
        local += o;
    }
    part[threadIdx.x] = local;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int q = 0; q < 256; ++q) {
            const int v = part[q];
            part[q] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int i = i0; i < i1; ++i) open[i] += part[threadIdx.x];
    __syncthreads();
    for (int i = threadIdx.x; i < N; i += 256) {
        const int l = row[i];
        out[i] = (l >= 0 && l < N) ? open[first[l]] : l;
    }
    if (threadIdx.x == 0) {
        out[N] = b.i;
        *out_f = b.f;
    }
}

hipError_t launch_best(const double *fitness, const int32_t *labels, int P, int N, int32_t *out,
                       double *out_f, hipStream_t s) {
    hipLaunchKernelGGL(k_best, dim3(1), dim3(256), 0, s, fitness, labels, P, N, out, out_f);
    return hipGetLastError();
}

}  // namespace pga
