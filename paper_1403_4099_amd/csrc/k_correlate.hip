// Correlation (Eq. 7 of Section 2.2.3) and the BF16 hi + lo split of C.
//
//   row stats : mean_i and s_i = sum_t (R_it - mean_i)^2 (two passes, FP64)
//   corr      : C_ij = sum_t x_it x_jt / sqrt(s_i s_j): FP64 MFMA Gram on 128 x 128
//               output tiles of the upper triangle (t split into slices), x =
//               R - mean staged through LDS; the slices added in order, C_ii =
//               1, clamp to [-1, 1], zero-variance stocks get 0 off the
//               diagonal, mirrored store
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

// ---- Gram matrix on FP64 MFMA ----------------------------------------------------
// G_ij = sum_t x_it x_jt over the upper triangle of 128 x 128 output tiles,
// each tile's t range split into S slices (gram_split: about one workgroup per
// CU), one workgroup per (tile, slice):
//   * the workgroup stages x of its 128 + 128 rows, 16 samples at a time, in
//     LDS (two buffers: the next chunk's global loads are in flight while the
//     current one is multiplied, 64 MFMAs per wave and chunk, enough to cover
//     a memory latency); x = R - mean for the correlation, the weighted
//     returns as they are for the EWMA covariance;
//   * wave w owns the 64 x 64 quadrant (w / 2, w % 2) of the tile: sixteen
//     16 x 16 blocks, each accumulated by v_mfma_f64_16x16x4_f64 (lane l
//     supplies A[l % 16][l / 16] and B[l / 16][l % 16]: row l % 16 of A and
//     column l % 16 of B at the samples t0 + 4 (l / 16) + e, e = 0..3, one per
//     MFMA, so both operands see the same t);
//   * the slice's 128 x 128 partial Gram goes to the workspace; a finish kernel
//     (one workgroup per 32 x 32 block of a tile) adds the S slices in slice
//     order (a fixed order: the result does not depend on timing), applies the
//     normalisation and writes the block and its mirror image through LDS,
//     both coalesced.
// A 128 x 128 tile moves half the bytes per flop of a 64 x 64 one: at N = 1024,
// T = 4096 the rows of R are read from the shared caches about 9 times in all.
typedef double gram_d4 __attribute__((ext_vector_type(4)));

constexpr int kGT = 128;                // output tile edge
constexpr int kGQ = 64;                 // quadrant edge of one wave
constexpr int kGK = 16;                 // samples per staged chunk
constexpr int kGPad = kGK + 2;          // LDS row stride (doubles): 16-byte aligned rows, spread banks
constexpr int kGMaxSplit = 16;

int gram_tiles(int N) {
    const int nt = (N + kGT - 1) / kGT;
    return nt * (nt + 1) / 2;
}

// Slices per tile for a given N (upper bound) and, with T known, the slices used:
// about 256 workgroups in all (one per CU), at most kGMaxSplit, and at least 64
// samples per slice. (Two per CU measured slower: the doubled partial traffic
// of the finish outweighs the second wave per SIMD.)
int gram_split_max(int N) {
    const int t = gram_tiles(N);
    int S = (256 + t / 2) / t;
    return S < 1 ? 1 : (S > kGMaxSplit ? kGMaxSplit : S);
}

int gram_split(int N, int T) {
    int S = gram_split_max(N);
    const int by_t = T / 64 > 1 ? T / 64 : 1;
    return S < by_t ? S : by_t;
}

size_t gram_ws_doubles(int N) { return (size_t)gram_tiles(N) * gram_split_max(N) * kGT * kGT; }

// Tile u of the upper triangle, row-major: (ti, tj) with ti <= tj.
__device__ __forceinline__ void gram_tile_ij(int u, int nt, int &ti, int &tj) {
    ti = 0;
    while (u >= nt - ti) {
        u -= nt - ti;
        ++ti;
    }
    tj = ti + u;
}

template <bool CENTER>
__global__ __launch_bounds__(256) void k_gram_mfma(const double *X, int N, int T, int64_t ld, const double *mu,
                                                   int nt, int tiles, int S, double *part) {
    __shared__ __align__(16) double sA[2][kGT * kGPad];
    __shared__ __align__(16) double sB[2][kGT * kGPad];
    const int total = tiles * S;
    const int unit = xcd_tile(blockIdx.x, total);           // each XCD: a contiguous range of units
    const int slice = unit / tiles, tile = unit - slice * tiles;
    int ti, tj;
    gram_tile_ij(tile, nt, ti, tj);
    const int i0 = ti * kGT, j0 = tj * kGT;
    const int per = ((T + S - 1) / S + kGK - 1) / kGK * kGK;  // samples per slice, whole chunks
    const int ts = slice * per;
    const int te = min(T, ts + per);

    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    // staging: thread t takes samples 2 (t % 8), +1 of rows t / 8 + 32 e (e = 0..3) of each
    // panel, so 8 threads read a row's 16-sample segment and a load instruction of a wave
    // covers eight rows
    const int srow = tid >> 3, scol = 2 * (tid & 7);
    // Loads take clamped (always valid) addresses and the value is zeroed afterwards where the row is
    // past N or the sample past the slice (a clamped address repeats an element of the same row or
    // of row N - 1, whose entries are discarded), so every load is issued unconditionally and
    // together with the others.
    double muA[4], muB[4];
    int rowA[4], rowB[4];
    uint32_t valid = 0;                                      // bit e: row e of A; bit 4 + e: of B
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const int ra = i0 + 32 * e + srow, rb = j0 + 32 * e + srow;
        rowA[e] = min(ra, N - 1);
        rowB[e] = min(rb, N - 1);
        muA[e] = CENTER ? mu[rowA[e]] : 0.0;
        muB[e] = CENTER ? mu[rowB[e]] : 0.0;
        valid |= (ra < N ? 1u : 0u) << e;
        valid |= (rb < N ? 1u : 0u) << (4 + e);
    }
    // The raw values are loaded first and only used when they are stored into LDS, after the
    // current chunk's MFMAs have been issued, so the loads' latency is hidden behind them.
    double va[4][2], vb[4][2];
    bool tin0 = false, tin1 = false;
    auto load = [&](int t0) {
        const int t = t0 + scol;
        tin0 = t < te;
        tin1 = t + 1 < te;
        const int tc0 = min(t, te - 1), tc1 = min(t + 1, te - 1);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            va[e][0] = X[(size_t)rowA[e] * ld + tc0];
            va[e][1] = X[(size_t)rowA[e] * ld + tc1];
            vb[e][0] = X[(size_t)rowB[e] * ld + tc0];
            vb[e][1] = X[(size_t)rowB[e] * ld + tc1];
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const bool a = (valid >> e) & 1u, b = (valid >> (4 + e)) & 1u;
            double *pa = &sA[buf][(32 * e + srow) * kGPad + scol];
            double *pb = &sB[buf][(32 * e + srow) * kGPad + scol];
            pa[0] = (tin0 && a) ? va[e][0] - muA[e] : 0.0;
            pa[1] = (tin1 && a) ? va[e][1] - muA[e] : 0.0;
            pb[0] = (tin0 && b) ? vb[e][0] - muB[e] : 0.0;
            pb[1] = (tin1 && b) ? vb[e][1] - muB[e] : 0.0;
        }
    };

    const int qr = wave >> 1, qc = wave & 1;
    const int m = lane & 15, kq = lane >> 4;
    gram_d4 acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = gram_d4{0.0, 0.0, 0.0, 0.0};

    int buf = 0;
    if (ts < te) {
        load(ts);
        store(0);
    }
    __syncthreads();
    for (int t0 = ts; t0 < te; t0 += kGK) {
        const bool more = t0 + kGK < te;
        if (more) load(t0 + kGK);
        const double *A = sA[buf];
        const double *B = sB[buf];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            double xa[4], xb[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
                xa[a] = A[(kGQ * qr + 16 * a + m) * kGPad + 4 * kq + e];
                xb[a] = B[(kGQ * qc + 16 * a + m) * kGPad + 4 * kq + e];
            }
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[a], xb[b], acc[a][b], 0, 0, 0);
        }
        if (more) store(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // Where each accumulator register sits in its 16 x 16 block is read off the hardware: one
    // MFMA with A[i][0] = i, B[0][j] = 1 (zero for k > 0) gives every register its row i, one with
    // A[i][0] = 1, B[0][j] = j its column j (small integers, exact in FP64). On this GPU register r
    // of lane l holds D[l / 16 + 4 r][l % 16].
    const double idx = kq == 0 ? (double)m : 0.0, one = kq == 0 ? 1.0 : 0.0;
    const gram_d4 zero = {0.0, 0.0, 0.0, 0.0};
    const gram_d4 rowv = __builtin_amdgcn_mfma_f64_16x16x4f64(idx, one, zero, 0, 0, 0);
    const gram_d4 colv = __builtin_amdgcn_mfma_f64_16x16x4f64(one, idx, zero, 0, 0, 0);
    double *out = part + ((size_t)slice * tiles + tile) * (kGT * kGT);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int ri = (int)rowv[r], ci = (int)colv[r];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b)
                out[(kGQ * qr + 16 * a + ri) * kGT + kGQ * qc + 16 * b + ci] = acc[a][b][r];
    }
}

// One workgroup per 32 x 32 block of a tile (blockIdx.x = 16 tile + block): writes value
// f(i, j, g) of every element of the block at (i, j) and, off the diagonal, at (j, i), both
// row-wise through an LDS transpose. g is the sum of the element's S slice partials in slice
// order; a thread issues the partial loads of its 4 elements together (one memory latency for
// all). Only i <= j is written directly and i < j mirrored, so the blocks below the diagonal of
// a diagonal tile write nothing.
constexpr int kGE = 32;
template <class F>
__device__ __forceinline__ void gram_emit(const double *part, int N, int nt, int tiles, int S, double *dst, F f) {
    __shared__ double tr[kGE][kGE + 1];
    const int tile = blockIdx.x >> 4, blk = blockIdx.x & 15;
    int ti, tj;
    gram_tile_ij(tile, nt, ti, tj);
    const int r0 = kGE * (blk >> 2), c0 = kGE * (blk & 3);   // within the tile
    if (ti == tj && r0 > c0) return;                          // uniform: every element has i > j
    const int i0 = ti * kGT + r0, j0 = tj * kGT + c0;
    const size_t sstride = (size_t)tiles * (kGT * kGT);
    const double *base = part + (size_t)tile * (kGT * kGT);
    double g[4][kGMaxSplit];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + 256 * u, r = e / kGE, c = e % kGE;
        const double *p = base + (size_t)(r0 + r) * kGT + c0 + c;
#pragma unroll
        for (int s = 0; s < kGMaxSplit; ++s) g[u][s] = s < S ? p[(size_t)s * sstride] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + 256 * u, r = e / kGE, c = e % kGE;
        const int i = i0 + r, j = j0 + c;
        double sum = 0.0;
#pragma unroll
        for (int s = 0; s < kGMaxSplit; ++s)
            if (s < S) sum += g[u][s];
        double v = 0.0;
        if (i < N && j < N && i <= j) {
            v = f(i, j, sum);
            dst[(size_t)i * N + j] = v;
        }
        tr[c][r] = v;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = threadIdx.x + 256 * u, r = e / kGE, c = e % kGE;   // destination row j0 + r, column i0 + c
        const int j = j0 + r, i = i0 + c;
        if (i < N && j < N && i < j) dst[(size_t)j * N + i] = tr[r][c];
    }
}

__global__ __launch_bounds__(256) void k_corr_finish(const double *part, int N, int nt, int tiles, int S,
                                                     const double *ss, double *C) {
    gram_emit(part, N, nt, tiles, S, C, [&](int i, int j, double g) {
        if (i == j) return 1.0;
        const double a = ss[i], b = ss[j];
        if (a == 0.0 || b == 0.0) return 0.0;
        return fmin(1.0, fmax(-1.0, g / sqrt(a * b)));
    });
}

hipError_t launch_corr(const double *R, int N, int T, int64_t ld, const double *mu, const double *ss,
                       double *C, double *part, hipStream_t s) {
    const int nt = (N + kGT - 1) / kGT, tiles = gram_tiles(N), S = gram_split(N, T);
    hipLaunchKernelGGL(k_gram_mfma<true>, dim3(tiles * S), dim3(256), 0, s, R, N, T, ld, mu, nt, tiles, S, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_corr_finish, dim3(16 * tiles), dim3(256), 0, s, part, N, nt, tiles, S, ss, C);
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
//          the upper triangle (the MFMA Gram of the correlation), mirrored;
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

__global__ __launch_bounds__(256) void k_ewma_finish(const double *part, int N, int nt, int tiles, int S,
                                                     double decay, int reset, double *Sm) {
    gram_emit(part, N, nt, tiles, S, Sm, [&](int i, int j, double g) {
        return reset ? g : fma(decay, Sm[(size_t)i * N + j], g);
    });
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
                       double *C, double *X, double *part, int32_t *status, hipStream_t s) {
    hipLaunchKernelGGL(k_ewma_prep, dim3((T + 255) / 256), dim3(256), 0, s, R, N, T, ld, lam, market, X);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int nt = (N + kGT - 1) / kGT, tiles = gram_tiles(N), Sp = gram_split(N, T);
    hipLaunchKernelGGL(k_gram_mfma<false>, dim3(tiles * Sp), dim3(256), 0, s, X, N, T, (int64_t)T, nullptr, nt,
                       tiles, Sp, part);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(k_ewma_finish, dim3(16 * tiles), dim3(256), 0, s, part, N, nt, tiles, Sp,
                       pow(lam, (double)T), reset, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t nn = (int64_t)N * N;
    hipLaunchKernelGGL(k_ewma_norm, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0, s, S, N, C, status);
    return hipGetLastError();
}

}  // namespace pga
