// Fitness kernels: the Giada-Marsili likelihood L_c (Eq. 8) of a population,
// from n_s (Eq. 5) and c_s (Eq. 6).
//
// Split into two launches:
//   pair-sum  w_pj = sum_{i<j} [s_pi = s_pj] C_ij  for every individual p and
//             stock j (the O(N^2) part; FP64 VALU or BF16x2 MFMA form);
//   finish    per individual: n_s by an LDS histogram, c_s = sum_{j in s}
//             (C_jj + 2 w_pj) grouped exactly in 64-bit fixed point, then the
//             FP64 log terms and a fixed-order block reduction.
// Nothing here uses floating-point atomics, so every result is a pure
// function of (C, labels): reruns and batching cannot change a bit.
#include "pga_internal.hpp"

#include <math.h>

namespace pga {

// ---------------------------------------------------------------------------
// Descriptor upload for single-instance calls: the descriptor and prefix
// tables travel as kernel arguments, so no host buffer has to outlive the call.
struct DescBlob {
    InstDesc d;
    int32_t prefix[6];   // {0, fp64 tiles}, {0, mfma tiles}, {0, P}
};

__global__ void k_write_desc(DescBlob b, InstDesc *dst, int32_t *prefix) {
    if (threadIdx.x == 0) *dst = b.d;
    if (threadIdx.x < 6) prefix[threadIdx.x] = b.prefix[threadIdx.x];
}

hipError_t launch_write_desc(const InstDesc &d, InstDesc *dst, int32_t *prefix, hipStream_t s) {
    DescBlob b;
    b.d = d;
    b.prefix[0] = 0;
    b.prefix[1] = fp64_tiles(d.N, d.P);
    b.prefix[2] = 0;
    b.prefix[3] = mfma_tiles(d.N, d.P);
    b.prefix[4] = 0;
    b.prefix[5] = d.P;
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(64), 0, s, b, dst, prefix);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 pair-sum. One workgroup = 64 consecutive stocks j (one per lane) x 64
// individuals (16 per wave). Each lane keeps its 16 labels s_pj and 16 FP64
// accumulators in registers and walks the rows i < j of its column: the
// column entry C_ij is loaded once (coalesced across the wave, L2-resident)
// and reused by 16 individuals; the row labels s_pi are staged per 64-row
// chunk in LDS, transposed so one 16-byte broadcast read serves 4
// individuals. Per (pair, individual): compare, select 1.0/0.0, FMA.
// Symmetry: only i < j is visited; the finish kernel doubles it and adds C_jj.
__global__ __launch_bounds__(256) void k_pairsum_fp64(Tables t, int parity) {
    constexpr int B = kFp64B;
    __shared__ int4 lab_s[kFp64Waves][64][B / 4];

    const int tile = blockIdx.x;
    const int k = find_inst(t.tiles_fp64, t.n_inst, tile);
    const InstDesc &d = t.desc[k];
    const int N = d.N, P = d.P;
    const int local = tile - t.tiles_fp64[k];
    const int n_jb = (N + kFp64Cols - 1) / kFp64Cols;
    const int jb = n_jb - 1 - (local % n_jb);          // heaviest column blocks first
    const int pb = local / n_jb;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int j = jb * kFp64Cols + lane;
    const bool jok = j < N;
    const int pbase = pb * kFp64Inds + wave * B;
    const int32_t *__restrict__ labels = d.pop[parity];
    const double *__restrict__ C = d.C;

    int lj[B];
    double acc[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int p = pbase + b;
        lj[b] = (jok && p < P) ? labels[(size_t)p * N + j] : (int)0x80000000;
        acc[b] = 0.0;
    }

    const int iend = min(jb * kFp64Cols + kFp64Cols, N);
    for (int i0 = 0; i0 < iend; i0 += 64) {
        {
            const int ir = i0 + lane;
            int v[B];
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int p = pbase + b;
                v[b] = (ir < N && p < P) ? labels[(size_t)p * N + ir] : (int)0x80000001;
            }
#pragma unroll
            for (int q = 0; q < B / 4; ++q)
                lab_s[wave][lane][q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
        }
        __syncthreads();
        const int rows = min(64, iend - i0);
#pragma unroll 4
        for (int r = 0; r < rows; ++r) {
            const int i = i0 + r;
            const double c = (jok && i < j) ? C[(size_t)i * N + j] : 0.0;
#pragma unroll
            for (int q = 0; q < B / 4; ++q) {
                const int4 rl = lab_s[wave][r][q];
                acc[4 * q + 0] = fma(rl.x == lj[4 * q + 0] ? 1.0 : 0.0, c, acc[4 * q + 0]);
                acc[4 * q + 1] = fma(rl.y == lj[4 * q + 1] ? 1.0 : 0.0, c, acc[4 * q + 1]);
                acc[4 * q + 2] = fma(rl.z == lj[4 * q + 2] ? 1.0 : 0.0, c, acc[4 * q + 2]);
                acc[4 * q + 3] = fma(rl.w == lj[4 * q + 3] ? 1.0 : 0.0, c, acc[4 * q + 3]);
            }
        }
        __syncthreads();
    }
    if (jok) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            if (p < P) d.wsum[(size_t)p * N + j] = acc[b];
        }
    }
}

hipError_t launch_pairsum_fp64(Tables t, int total_tiles, int parity, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairsum_fp64, dim3(total_tiles), dim3(256), 0, s, t, parity);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finish: one workgroup per individual.
//   1. validity of labels, v_j = C_jj + 2 w_j, max |v_j|;
//   2. n_s and sum_{j in s} v_j by integer LDS atomics, v_j scaled by 2^sc and
//      rounded to int64 (sc chosen per individual so N max|v| 2^sc < 2^62:
//      the integer sums are exact and order-free, error <= n_s 2^-(sc+1));
//   3. per label s with n_s > 1: c_s, domain check, the two FP64 log terms
//      of Eq. 8 in literal form; per-thread sums in ascending s, then a
//      fixed tree over the workgroup.
__device__ __forceinline__ double block_sum_fixed(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(256) void k_finish(Tables t, int parity, int32_t *status) {
    extern __shared__ unsigned char smem[];
    __shared__ double red[256];
    __shared__ int flags;

    const int g = blockIdx.x;
    const int k = find_inst(t.inds, t.n_inst, g);
    const InstDesc &d = t.desc[k];
    const int N = d.N;
    const int p = g - t.inds[k];
    const int32_t *__restrict__ lab = d.pop[parity] + (size_t)p * N;
    const double *__restrict__ w = d.wsum + (size_t)p * N;
    const double *__restrict__ C = d.C;
    long long *csum = (long long *)smem;
    int *cnt = (int *)(smem + sizeof(long long) * (size_t)N);

    if (threadIdx.x == 0) flags = 0;
    __syncthreads();
    int bad = 0;
    double mx = 0.0;
    for (int j = threadIdx.x; j < N; j += 256) {
        const int l = lab[j];
        if (l < 0 || l >= N) bad |= 1;
        const double v = C[(size_t)j * N + j] + 2.0 * w[j];
        if (!isfinite(v)) bad |= 2;
        else mx = fmax(mx, fabs(v));
    }
    if (bad) atomicOr(&flags, bad);
    // max over the workgroup (order-free)
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
        __syncthreads();
    }
    mx = red[0];
    const int fl = flags;
    __syncthreads();

    if (fl) {
        if (threadIdx.x == 0) {
            d.fitness[p] = -INFINITY;
            if (status) {
                if (fl & 1) atomicAdd(&status[PGA_ST_LABEL], 1);
                atomicAdd(&status[PGA_ST_NONFINITE], 1);
            }
        }
        if (d.n_s_out)
            for (int s = threadIdx.x; s < N; s += 256) d.n_s_out[(size_t)p * N + s] = 0;
        if (d.c_s_out)
            for (int s = threadIdx.x; s < N; s += 256) d.c_s_out[(size_t)p * N + s] = 0.0;
        return;
    }

    for (int s = threadIdx.x; s < N; s += 256) {
        csum[s] = 0;
        cnt[s] = 0;
    }
    int sc = 0;
    if (mx > 0.0) {
        int e;
        frexp(mx * (double)N, &e);   // N max|v| < 2^e
        sc = 61 - e;
    }
    __syncthreads();
    for (int j = threadIdx.x; j < N; j += 256) {
        const int l = lab[j];
        const double v = C[(size_t)j * N + j] + 2.0 * w[j];
        const long long q = llrint(ldexp(v, sc));
        atomicAdd(&cnt[l], 1);
        atomicAdd((unsigned long long *)&csum[l], (unsigned long long)q);
    }
    __syncthreads();

    double L = 0.0;
    int nbad = 0;
    for (int s = threadIdx.x; s < N; s += 256) {
        const int n = cnt[s];
        const double c = ldexp((double)csum[s], -sc);
        if (d.n_s_out) d.n_s_out[(size_t)p * N + s] = n;
        if (d.c_s_out) d.c_s_out[(size_t)p * N + s] = c;
        if (n > 1) {
            const double nd = (double)n;
            const double n2 = nd * nd;
            if (!(c > 0.0 && c < n2)) {
                nbad += 1;
            } else {
                L += log(nd / c) + (nd - 1.0) * log((n2 - nd) / (n2 - c));
            }
        }
    }
    const double Ltot = block_sum_fixed(L, red);
    const double badtot = block_sum_fixed((double)nbad, red);
    if (threadIdx.x == 0) {
        if (badtot > 0.0) {
            d.fitness[p] = -INFINITY;
            if (status) {
                atomicAdd(&status[PGA_ST_DOMAIN], (int)badtot);
                atomicAdd(&status[PGA_ST_NONFINITE], 1);
            }
        } else {
            d.fitness[p] = 0.5 * Ltot;
        }
    }
}

hipError_t launch_finish(Tables t, int total_inds, int max_n, int parity, int32_t *status,
                         hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    const size_t lds = (size_t)max_n * (sizeof(long long) + sizeof(int));
    hipLaunchKernelGGL(k_finish, dim3(total_inds), dim3(256), lds, s, t, parity, status);
    return hipGetLastError();
}

}  // namespace pga
