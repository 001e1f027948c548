// Correlation (Eq. 7 of Section 2.2.3) and the BF16 hi + lo split of C.
//
//   row stats : mean_i and s_i = sum_t (R_it - mean_i)^2 (two passes, FP64)
//   corr      : C_ij = sum_t x_it x_jt / sqrt(s_i s_j) on 64 x 64 output tiles
//               of the upper triangle, x = R - mean staged through LDS,
//               FP64 FMA in ascending t; mirrored store, C_ii = 1, clamp to
//               [-1, 1], zero-variance stocks get 0 off the diagonal
//   split     : hi = bf16(C), lo = bf16(C - hi), round to nearest even from
//               FP64, zero padding up to the 32-aligned leading dimension
#include "pga_internal.hpp"

#include <math.h>

namespace pga {

__global__ __launch_bounds__(256) void k_row_stats(const double *R, int T, int64_t ld, double *mu,
                                                   double *ss, int32_t *status) {
    __shared__ double red[256];
    const int i = blockIdx.x;
    const double *__restrict__ row = R + (size_t)i * ld;
    double s = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) s += row[t];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    const double m = red[0] / (double)T;
    __syncthreads();
    double q = 0.0;
    for (int t = threadIdx.x; t < T; t += 256) {
        const double x = row[t] - m;
        q = fma(x, x, q);
    }
    red[threadIdx.x] = q;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        mu[i] = m;
        ss[i] = red[0];
        if (red[0] == 0.0 && status) atomicAdd(&status[PGA_ST_ZEROVAR], 1);
    }
}

hipError_t launch_row_stats(const double *R, int N, int T, int64_t ld, double *mu, double *ss,
                            int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_row_stats, dim3(N), dim3(256), 0, s, R, T, ld, mu, ss, status);
    return hipGetLastError();
}

// 64 x 64 output tile per workgroup; thread (tx, ty) owns rows i0 + 4ty..+3
// and columns j0 + 4tx..+3. K loop over t in chunks of 16 through LDS.
constexpr int kCT = 64, kCK = 16;

__global__ __launch_bounds__(256) void k_corr(const double *R, int N, int T, int64_t ld,
                                              const double *mu, const double *ss, double *C) {
    __shared__ double As[kCK][kCT + 1];
    __shared__ double Bs[kCK][kCT + 1];
    const int ti = blockIdx.y, tj = blockIdx.x;
    if (ti > tj) return;
    const int i0 = ti * kCT, j0 = tj * kCT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;

    double acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

    for (int t0 = 0; t0 < T; t0 += kCK) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int idx = threadIdx.x + 256 * e;   // 0..1023
            const int r = idx >> 4, kk = idx & 15;
            const int t = t0 + kk;
            const int gi = i0 + r, gj = j0 + r;
            As[kk][r] = (gi < N && t < T) ? R[(size_t)gi * ld + t] - mu[gi] : 0.0;
            Bs[kk][r] = (gj < N && t < T) ? R[(size_t)gj * ld + t] - mu[gj] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kCK; ++kk) {
            double a[4], b[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                a[q] = As[kk][4 * ty + q];
                b[q] = Bs[kk][4 * tx + q];
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = 0; y < 4; ++y) acc[x][y] = fma(a[x], b[y], acc[x][y]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int i = i0 + 4 * ty + x;
        if (i >= N) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int j = j0 + 4 * tx + y;
            if (j >= N || j < i) continue;
            double v;
            if (i == j) {
                v = 1.0;
            } else if (ss[i] == 0.0 || ss[j] == 0.0) {
                v = 0.0;
            } else {
                v = acc[x][y] / sqrt(ss[i] * ss[j]);
                v = fmin(1.0, fmax(-1.0, v));
            }
            C[(size_t)i * N + j] = v;
            C[(size_t)j * N + i] = v;
        }
    }
}

hipError_t launch_corr(const double *R, int N, int T, int64_t ld, const double *mu, const double *ss,
                       double *C, hipStream_t s) {
    const int nt = (N + kCT - 1) / kCT;
    hipLaunchKernelGGL(k_corr, dim3(nt, nt), dim3(256), 0, s, R, N, T, ld, mu, ss, C);
    return hipGetLastError();
}

// Round an FP64 value to the nearest bfloat16 value (ties to even) in one
// step, by integer arithmetic on the FP64 bit pattern: keep the top 7 of
// the 52 stored mantissa bits with round-half-even on the 45 dropped bits.
// Below 2^-126 bfloat16 is subnormal with spacing 2^-133: there the value is
// scaled by 2^133, rounded to an integer (rint is half-even) and scaled back.
__device__ __forceinline__ double bf16_round(double x) {
    if (x == 0.0 || !isfinite(x)) return x;
    unsigned long long u = (unsigned long long)__double_as_longlong(x);
    const int bexp = (int)((u >> 52) & 0x7FF);
    if (bexp >= 1023 - 126) {
        const unsigned long long lsb = (u >> 45) & 1ull;
        u += (1ull << 44) - 1ull + lsb;
        u &= ~((1ull << 45) - 1ull);
        return __longlong_as_double((long long)u);
    }
    return rint(x * 0x1p133) * 0x1p-133;
}

__device__ __forceinline__ uint16_t bf16_bits(double r) {
    return (uint16_t)(__float_as_uint((float)r) >> 16);
}

__global__ __launch_bounds__(256) void k_split(const double *C, int N, int ld, uint16_t *hi, uint16_t *lo) {
    const size_t total = (size_t)ld * ld;
    for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (size_t)gridDim.x * 256) {
        const int i = (int)(e / ld), j = (int)(e % ld);
        const double v = (i < N && j < N) ? C[(size_t)i * N + j] : 0.0;
        const double h = bf16_round(v);
        const double l = bf16_round(v - h);
        hi[e] = bf16_bits(h);
        lo[e] = bf16_bits(l);
    }
}

hipError_t launch_split(const double *C, int N, uint16_t *hi, uint16_t *lo, hipStream_t s) {
    const int ld = split_ld(N);
    const size_t total = (size_t)ld * ld;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_split, dim3(blocks), dim3(256), 0, s, C, N, ld, hi, lo);
    return hipGetLastError();
}

}  // namespace pga
