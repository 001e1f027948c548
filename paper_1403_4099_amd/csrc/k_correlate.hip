// Correlation (Eq. 7 of Section 2.2.3) and the BF16 hi + lo split of C.
//
//   row stats : mean_i and s_i = sum_t (R_it - mean_i)^2 (two passes, FP64)
//   corr      : C_ij = sum_t x_it x_jt / sqrt(s_i s_j) on 64 x 64 output tiles
//               of the upper triangle, x = R - mean staged through LDS,
//               FP64 FMA in ascending t; mirrored store, C_ii = 1, clamp to
//               [-1, 1], zero-variance stocks get 0 off the diagonal
//   split     : hi = bf16(C), lo = bf16(C - hi), round to nearest even from
//               FP64, zero padding up to the 32-aligned leading dimension
//   ewma      : online exponentially weighted correlation with the market
//               mode removed (pre-processing step before the path)
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
// and columns j0 + 4tx..+3. K loop over t in chunks of 16 through LDS;
// x(g, t) gives the (already centred or weighted) value of row g at time t.
constexpr int kCT = 64, kCK = 16;

template <class X>
__device__ __forceinline__ void gram_tile(X x, int N, int T, int i0, int j0, double (&acc)[4][4]) {
    __shared__ double As[kCK][kCT + 1];
    __shared__ double Bs[kCK][kCT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
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
            As[kk][r] = (gi < N && t < T) ? x(gi, t) : 0.0;
            Bs[kk][r] = (gj < N && t < T) ? x(gj, t) : 0.0;
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
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_corr(const double *R, int N, int T, int64_t ld,
                                              const double *mu, const double *ss, double *C) {
    const int ti = blockIdx.y, tj = blockIdx.x;
    if (ti > tj) return;
    const int i0 = ti * kCT, j0 = tj * kCT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
    gram_tile([&](int g, int t) { return R[(size_t)g * ld + t] - mu[g]; }, N, T, i0, j0, acc);
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

// ---- online EWMA correlation (Section 4.2.5 pre-processing) ------------------
// The recursion S <- lambda S + (1 - lambda) x_t x_t^T over t = 0 .. T-1 is
// S <- lambda^T S + sum_t w_t x_t x_t^T with w_t = (1 - lambda) lambda^(T-1-t):
//   prep : x_it = sqrt(w_t) (R_it - m_t), m_t the equal-weight market return
//          (sum over i in ascending order, / N) or 0; one thread per t;
//   gram : S_ij <- lambda^T S_ij + sum_t x_it x_jt on the 64 x 64 tiles of
//          the upper triangle (same FP64 tile as the correlation), mirrored;
//   norm : C_ij = S_ij / sqrt(S_ii S_jj), clamp, C_ii = 1, zero variance -> 0.
__global__ __launch_bounds__(256) void k_ewma_prep(const double *R, int N, int T, int64_t ld, double lam,
                                                   int market, double *X) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= T) return;
    double m = 0.0;
    if (market) {
        for (int i = 0; i < N; ++i) m += R[(size_t)i * ld + t];
        m /= (double)N;
    }
    const double sw = sqrt((1.0 - lam) * pow(lam, (double)(T - 1 - t)));
    for (int i = 0; i < N; ++i) X[(size_t)i * T + t] = sw * (R[(size_t)i * ld + t] - m);
}

__global__ __launch_bounds__(256) void k_ewma_gram(const double *X, int N, int T, double decay, int reset,
                                                   double *S) {
    const int ti = blockIdx.y, tj = blockIdx.x;
    if (ti > tj) return;
    const int i0 = ti * kCT, j0 = tj * kCT;
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    double acc[4][4];
    gram_tile([&](int g, int t) { return X[(size_t)g * T + t]; }, N, T, i0, j0, acc);
#pragma unroll
    for (int x = 0; x < 4; ++x) {
        const int i = i0 + 4 * ty + x;
        if (i >= N) continue;
#pragma unroll
        for (int y = 0; y < 4; ++y) {
            const int j = j0 + 4 * tx + y;
            if (j >= N || j < i) continue;
            const double v = reset ? acc[x][y] : fma(decay, S[(size_t)i * N + j], acc[x][y]);
            S[(size_t)i * N + j] = v;
            S[(size_t)j * N + i] = v;
        }
    }
}

__global__ __launch_bounds__(256) void k_ewma_norm(const double *S, int N, double *C, int32_t *status) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= (int64_t)N * N) return;
    const int i = (int)(e / N), j = (int)(e - (int64_t)i * N);
    const double a = S[(size_t)i * N + i], b = S[(size_t)j * N + j];
    double v;
    if (i == j) {
        v = 1.0;
        if (a == 0.0 && status) atomicAdd(&status[PGA_ST_ZEROVAR], 1);
    } else if (a == 0.0 || b == 0.0) {
        v = 0.0;
    } else {
        v = fmin(1.0, fmax(-1.0, S[(size_t)i * N + j] / sqrt(a * b)));
    }
    C[e] = v;
}

hipError_t launch_ewma(const double *R, int N, int T, int64_t ld, double lam, int reset, int market, double *S,
                       double *C, double *X, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_ewma_prep, dim3((T + 255) / 256), dim3(256), 0, s, R, N, T, ld, lam, market, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nt = (N + kCT - 1) / kCT;
    hipLaunchKernelGGL(k_ewma_gram, dim3(nt, nt), dim3(256), 0, s, X, N, T, pow(lam, (double)T), reset, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(k_ewma_norm, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, S, N, C, status);
    return hipGetLastError();
}

}  // namespace pga
