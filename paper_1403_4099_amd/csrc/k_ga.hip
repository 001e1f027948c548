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
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int N = d.N;
    const int p = g - t.inds[k];
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

__global__ __launch_bounds__(256) void k_rank(Tables t, int gen_off) {
    __shared__ double rf[256];
    __shared__ int ri[256];
    const InstDesc &d = t.desc[blockIdx.x];
    const int P = d.P, E = d.E;
    const double *__restrict__ f = d.fitness;

    Cand prev{0.0, -1};
    int argbest = 0;
    const int rounds = E > 1 ? E : 1;
    for (int r = 0; r < rounds; ++r) {
        Cand c{0.0, -1};
        for (int p = threadIdx.x; p < P; p += 256) {
            const double fp = f[p];
            if (prev.i >= 0 && !ranks_before(prev.f, prev.i, fp, p)) continue;
            if (c.i < 0 || ranks_before(fp, p, c.f, c.i)) c = Cand{fp, p};
        }
        const Cand b = block_best(c, rf, ri);
        if (r == 0) argbest = b.i;
        if (r < E && threadIdx.x == 0) d.elite[r] = b.i;
        prev = b;
    }
    if (d.stats) {
        double sum = 0.0, ninv = 0.0;
        for (int p = threadIdx.x; p < P; p += 256) {
            const double fp = f[p];
            if (isfinite(fp)) sum += fp;
            else ninv += 1.0;
        }
        rf[threadIdx.x] = sum;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) rf[threadIdx.x] += rf[threadIdx.x + w];
            __syncthreads();
        }
        const double total = rf[0];
        __syncthreads();
        rf[threadIdx.x] = ninv;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) rf[threadIdx.x] += rf[threadIdx.x + w];
            __syncthreads();
        }
        const double inv = rf[0];
        if (threadIdx.x == 0) {
            double *row = d.stats + 4 * (size_t)gen_off;
            const double nfin = (double)P - inv;
            row[0] = f[argbest];
            row[1] = nfin > 0.0 ? total / nfin : -INFINITY;
            row[2] = inv;
            row[3] = (double)argbest;
        }
    }
}

hipError_t launch_rank(Tables t, int gen_off, hipStream_t s) {
    hipLaunchKernelGGL(k_rank, dim3(t.n_inst), dim3(256), 0, s, t, gen_off);
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

__global__ __launch_bounds__(256) void k_breed(Tables t, int parity, int gen_off) {
    const int g = blockIdx.x;
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int N = d.N, P = d.P, E = d.E;
    const int c = g - t.inds[k];
    const int32_t *__restrict__ src = d.pop[parity];
    int32_t *__restrict__ out = d.pop[parity ^ 1] + (size_t)c * N;

    if (c < E) {
        const int32_t *__restrict__ e = src + (size_t)d.elite[c] * N;
        for (int j = threadIdx.x; j < N; j += 256) out[j] = e[j];
        return;
    }
    const uint32_t gen = d.gen0 + (uint32_t)gen_off;
    const double *__restrict__ f = d.fitness;
    const U4 sel = draw(0u, (uint32_t)c, gen, kTagSel, d.inst_id, d.seed);
    const int A = tournament2(f, (int)scale_u32(sel.x, (uint32_t)P), (int)scale_u32(sel.y, (uint32_t)P));
    const int B = tournament2(f, (int)scale_u32(sel.z, (uint32_t)P), (int)scale_u32(sel.w, (uint32_t)P));
    const bool cross = draw(0u, (uint32_t)c, gen, kTagXov, d.inst_id, d.seed).x < d.p_cross;
    const int32_t *__restrict__ ra = src + (size_t)A * N;
    const int32_t *__restrict__ rb = src + (size_t)B * N;
    const uint32_t pm = d.p_mut;

    const int npair = (N + 1) >> 1;
    for (int jp = threadIdx.x; jp < npair; jp += 256) {
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

hipError_t launch_breed(Tables t, int total_inds, int parity, int gen_off, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_breed, dim3(total_inds), dim3(256), 0, s, t, parity, gen_off);
    return hipGetLastError();
}

// After an odd number of generations the population sits in pop[1]; copy it
// back so the caller always finds the result in the buffer it passed as pop.
__global__ __launch_bounds__(256) void k_copy_back(Tables t) {
    const int g = blockIdx.x;
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int N = d.N;
    const int p = g - t.inds[k];
    const int32_t *__restrict__ a = d.pop[1] + (size_t)p * N;
    int32_t *__restrict__ b = d.pop[0] + (size_t)p * N;
    for (int j = threadIdx.x; j < N; j += 256) b[j] = a[j];
}

hipError_t launch_copy_back(Tables t, int total_inds, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_back, dim3(total_inds), dim3(256), 0, s, t);
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
