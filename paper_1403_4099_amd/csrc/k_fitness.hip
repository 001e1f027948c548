// Fitness kernels: the Giada-Marsili likelihood L_c (Eq. 8) of a population,
// from n_s (Eq. 5) and c_s (Eq. 6).
//
// Split into two launches:
//   pair-sum  v_pj = C_jj + 2 sum_{i<j} [s_pi = s_pj] C_ij for every
//             individual p and stock j (the O(N^2) part; FP64 VALU form here,
//             BF16x2 MFMA form in k_mfma.hip);
//   finish    per individual: n_s by an LDS histogram, c_s = sum_{j in s} v_pj
//             grouped exactly in 64-bit fixed point, then the FP64 log terms
//             and a fixed-order wave reduction.
// Nothing here uses floating-point atomics, so every result is a pure
// function of (C, labels): reruns and batching cannot change a bit.
#include "pga_internal.hpp"

#include <math.h>

#include <type_traits>

namespace pga {

// ---------------------------------------------------------------------------
// Descriptor upload for single-instance calls: the descriptor and prefix
// tables travel as kernel arguments, so no host buffer has to outlive the call.
struct DescBlob {
    InstDesc d;
    int32_t prefix[4];   // {0, tiles}, {0, P}; the route list counters follow, zeroed
};

__global__ void k_write_desc(DescBlob b, InstDesc *dst, int32_t *prefix) {
    if (threadIdx.x == 0) *dst = b.d;
    if (threadIdx.x < 4) prefix[threadIdx.x] = b.prefix[threadIdx.x];
    for (int i = threadIdx.x; i < kListCounters; i += blockDim.x) prefix[4 + i] = 0;
}

hipError_t launch_write_desc(const InstDesc &d, int32_t tiles, InstDesc *dst, int32_t *prefix, hipStream_t s) {
    DescBlob b;
    b.d = d;
    b.prefix[0] = 0;
    b.prefix[1] = tiles;
    b.prefix[2] = 0;
    b.prefix[3] = d.P;
    hipLaunchKernelGGL(k_write_desc, dim3(1), dim3(256), 0, s, b, dst, prefix);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP64 pair-sum. One workgroup = 64 consecutive stocks j (one per lane) x 4B
// individuals (B = 8 or 16 per wave); the four waves are independent (no
// workgroup barrier). Each lane keeps its B labels s_pj and B FP64 accumulators in
// registers and walks the rows i < j of its column in chunks of 64 rows:
//   - C_ij is loaded once per (wave, row), coalesced across the wave, and
//     reused by B individuals; loads run one group of 4 rows ahead;
//   - the row labels s_pi of the wave's B individuals are staged per chunk in
//     a wave-private LDS buffer (transposed, so one 16-byte broadcast read
//     serves 4 individuals), double-buffered: the next chunk's labels are
//     fetched into registers while the current chunk is processed.
// Per (pair, individual): compare, masked FP64 add. Rows i >= j and rows
// past N contribute C = 0, so every chunk runs all 64 rows without branches.
// acc[b] += c on the lanes where row label r[b] equals lj[b], for the 8 or 16
// individuals of a wave: each compare writes a lane mask to an SGPR pair, the
// scalar unit narrows EXEC to it, and the FP64 add runs under that mask. Two
// vector instructions per (pair, individual); the scalar ones issue alongside
// other waves' vector work. Masks are made in two groups of 8, each group's
// compares under the full EXEC, which is restored before the block ends.
__device__ __forceinline__ void add_if_equal8(double *acc, const int *r, const int *lj, double c) {
    uint64_t m[8], sv;
    asm volatile(
        "s_mov_b64 %[sv], exec\n\t"
        "v_cmp_eq_u32_e64 %[m0], %[r0], %[l0]\n\t"
        "v_cmp_eq_u32_e64 %[m1], %[r1], %[l1]\n\t"
        "v_cmp_eq_u32_e64 %[m2], %[r2], %[l2]\n\t"
        "v_cmp_eq_u32_e64 %[m3], %[r3], %[l3]\n\t"
        "v_cmp_eq_u32_e64 %[m4], %[r4], %[l4]\n\t"
        "v_cmp_eq_u32_e64 %[m5], %[r5], %[l5]\n\t"
        "v_cmp_eq_u32_e64 %[m6], %[r6], %[l6]\n\t"
        "v_cmp_eq_u32_e64 %[m7], %[r7], %[l7]\n\t"
        "s_and_b64 exec, %[sv], %[m0]\n\t"
        "v_add_f64 %[a0], %[a0], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m1]\n\t"
        "v_add_f64 %[a1], %[a1], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m2]\n\t"
        "v_add_f64 %[a2], %[a2], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m3]\n\t"
        "v_add_f64 %[a3], %[a3], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m4]\n\t"
        "v_add_f64 %[a4], %[a4], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m5]\n\t"
        "v_add_f64 %[a5], %[a5], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m6]\n\t"
        "v_add_f64 %[a6], %[a6], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m7]\n\t"
        "v_add_f64 %[a7], %[a7], %[c]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [a0] "+v"(acc[0]), [a1] "+v"(acc[1]), [a2] "+v"(acc[2]), [a3] "+v"(acc[3]), [a4] "+v"(acc[4]), [a5] "+v"(acc[5]), [a6] "+v"(acc[6]), [a7] "+v"(acc[7]), [m0] "=&s"(m[0]), [m1] "=&s"(m[1]), [m2] "=&s"(m[2]), [m3] "=&s"(m[3]), [m4] "=&s"(m[4]), [m5] "=&s"(m[5]), [m6] "=&s"(m[6]), [m7] "=&s"(m[7]), [sv] "=&s"(sv)
        : [r0] "v"(r[0]), [r1] "v"(r[1]), [r2] "v"(r[2]), [r3] "v"(r[3]), [r4] "v"(r[4]), [r5] "v"(r[5]), [r6] "v"(r[6]), [r7] "v"(r[7]), [l0] "v"(lj[0]), [l1] "v"(lj[1]), [l2] "v"(lj[2]), [l3] "v"(lj[3]), [l4] "v"(lj[4]), [l5] "v"(lj[5]), [l6] "v"(lj[6]), [l7] "v"(lj[7]), [c] "v"(c)
        : "scc");
}

__device__ __forceinline__ void add_if_equal16(double *acc, const int *r, const int *lj, double c) {
    uint64_t m[8], sv;
    asm volatile(
        "s_mov_b64 %[sv], exec\n\t"
        "v_cmp_eq_u32_e64 %[m0], %[r0], %[l0]\n\t"
        "v_cmp_eq_u32_e64 %[m1], %[r1], %[l1]\n\t"
        "v_cmp_eq_u32_e64 %[m2], %[r2], %[l2]\n\t"
        "v_cmp_eq_u32_e64 %[m3], %[r3], %[l3]\n\t"
        "v_cmp_eq_u32_e64 %[m4], %[r4], %[l4]\n\t"
        "v_cmp_eq_u32_e64 %[m5], %[r5], %[l5]\n\t"
        "v_cmp_eq_u32_e64 %[m6], %[r6], %[l6]\n\t"
        "v_cmp_eq_u32_e64 %[m7], %[r7], %[l7]\n\t"
        "s_and_b64 exec, %[sv], %[m0]\n\t"
        "v_add_f64 %[a0], %[a0], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m1]\n\t"
        "v_add_f64 %[a1], %[a1], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m2]\n\t"
        "v_add_f64 %[a2], %[a2], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m3]\n\t"
        "v_add_f64 %[a3], %[a3], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m4]\n\t"
        "v_add_f64 %[a4], %[a4], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m5]\n\t"
        "v_add_f64 %[a5], %[a5], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m6]\n\t"
        "v_add_f64 %[a6], %[a6], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m7]\n\t"
        "v_add_f64 %[a7], %[a7], %[c]\n\t"
        "s_mov_b64 exec, %[sv]\n\t"
        "v_cmp_eq_u32_e64 %[m0], %[r8], %[l8]\n\t"
        "v_cmp_eq_u32_e64 %[m1], %[r9], %[l9]\n\t"
        "v_cmp_eq_u32_e64 %[m2], %[r10], %[l10]\n\t"
        "v_cmp_eq_u32_e64 %[m3], %[r11], %[l11]\n\t"
        "v_cmp_eq_u32_e64 %[m4], %[r12], %[l12]\n\t"
        "v_cmp_eq_u32_e64 %[m5], %[r13], %[l13]\n\t"
        "v_cmp_eq_u32_e64 %[m6], %[r14], %[l14]\n\t"
        "v_cmp_eq_u32_e64 %[m7], %[r15], %[l15]\n\t"
        "s_and_b64 exec, %[sv], %[m0]\n\t"
        "v_add_f64 %[a8], %[a8], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m1]\n\t"
        "v_add_f64 %[a9], %[a9], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m2]\n\t"
        "v_add_f64 %[a10], %[a10], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m3]\n\t"
        "v_add_f64 %[a11], %[a11], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m4]\n\t"
        "v_add_f64 %[a12], %[a12], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m5]\n\t"
        "v_add_f64 %[a13], %[a13], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m6]\n\t"
        "v_add_f64 %[a14], %[a14], %[c]\n\t"
        "s_and_b64 exec, %[sv], %[m7]\n\t"
        "v_add_f64 %[a15], %[a15], %[c]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [a0] "+v"(acc[0]), [a1] "+v"(acc[1]), [a2] "+v"(acc[2]), [a3] "+v"(acc[3]), [a4] "+v"(acc[4]), [a5] "+v"(acc[5]), [a6] "+v"(acc[6]), [a7] "+v"(acc[7]), [a8] "+v"(acc[8]), [a9] "+v"(acc[9]), [a10] "+v"(acc[10]), [a11] "+v"(acc[11]), [a12] "+v"(acc[12]), [a13] "+v"(acc[13]), [a14] "+v"(acc[14]), [a15] "+v"(acc[15]), [m0] "=&s"(m[0]), [m1] "=&s"(m[1]), [m2] "=&s"(m[2]), [m3] "=&s"(m[3]), [m4] "=&s"(m[4]), [m5] "=&s"(m[5]), [m6] "=&s"(m[6]), [m7] "=&s"(m[7]), [sv] "=&s"(sv)
        : [r0] "v"(r[0]), [r1] "v"(r[1]), [r2] "v"(r[2]), [r3] "v"(r[3]), [r4] "v"(r[4]), [r5] "v"(r[5]), [r6] "v"(r[6]), [r7] "v"(r[7]), [r8] "v"(r[8]), [r9] "v"(r[9]), [r10] "v"(r[10]), [r11] "v"(r[11]), [r12] "v"(r[12]), [r13] "v"(r[13]), [r14] "v"(r[14]), [r15] "v"(r[15]), [l0] "v"(lj[0]), [l1] "v"(lj[1]), [l2] "v"(lj[2]), [l3] "v"(lj[3]), [l4] "v"(lj[4]), [l5] "v"(lj[5]), [l6] "v"(lj[6]), [l7] "v"(lj[7]), [l8] "v"(lj[8]), [l9] "v"(lj[9]), [l10] "v"(lj[10]), [l11] "v"(lj[11]), [l12] "v"(lj[12]), [l13] "v"(lj[13]), [l14] "v"(lj[14]), [l15] "v"(lj[15]), [c] "v"(c)
        : "scc");
}

__device__ __forceinline__ double fp64_c(const double *__restrict__ C, int N, int i, int j) {
    return (i < j && j < N) ? gld(C + (size_t)i * N + j) : 0.0;
}

template <int B>
__global__ __launch_bounds__(256) void k_pairsum_fp64(Tables t, int parity, int order) {
    __shared__ int4 lab_s[kFp64Waves][2][64][B / 4];

    const int total = t.tiles[t.n_inst];                  // the grid may exceed it (capacity-sized graph)
    if ((int)blockIdx.x >= total) return;
    const int tile = order ? xcd_tile(blockIdx.x, total) : blockIdx.x;
    const int k = find_inst(t.tiles, t.n_inst, tile);
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;
    const int N = d.N, P = d.P;
    const int local = tile - t.tiles[k];
    const int n_jb = (N + kFp64Cols - 1) / kFp64Cols;
    const int n_pairs = (n_jb + 1) / 2;
    const TilePos tp = tile_pos(local, n_pairs, (P + kFp64Waves * B - 1) / (kFp64Waves * B), order);
    const int jp = tp.jp, pb = tp.pb;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform, kept scalar
    const int lane = threadIdx.x & 63;
    const int pbase = pb * (kFp64Waves * B) + wave * B;
    if (d.route) {                                   // wave-uniform: the waves share no barrier
        int any = 0;
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (pbase + b < P) any |= gld(d.route + pbase + b);
        if (!any) return;
    }
    const int32_t *__restrict__ labels = d.pop[parity];
    const double *__restrict__ C = d.C;
    const __amdgpu_buffer_rsrc_t c_r = __builtin_amdgcn_make_buffer_rsrc((void *)C, (short)0, 8 * N * N, kBufWord3);   // N <= 4096

    auto fetch_labels = [&](int i0, int *v) {
        const int ir = i0 + lane;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            v[b] = (ir < N && p < P) ? gld(labels + (size_t)p * N + ir) : (int)0x80000001;
        }
    };
    auto store_labels = [&](int buf, const int *v) {
#pragma unroll
        for (int q = 0; q < B / 4; ++q)
            lab_s[wave][buf][lane][q] = make_int4(v[4 * q], v[4 * q + 1], v[4 * q + 2], v[4 * q + 3]);
    };

    // The triangle is folded: column blocks n_jb-1-jp (jp + 1 ... n_jb chunks of rows) and
    // jp are done by the same workgroup, so every workgroup has n_jb + 1 chunks of work.
    for (int half = 0; half < 2; ++half) {
        const int jb = half == 0 ? n_jb - 1 - jp : jp;
        if (half == 1 && jb == n_jb - 1 - jp) break;       // middle block of an odd count: once
        const int j = jb * kFp64Cols + lane;
        const bool jok = j < N;

        int lj[B];
        double acc[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            lj[b] = (jok && p < P) ? gld(labels + (size_t)p * N + j) : (int)0x80000000;
            acc[b] = 0.0;
        }

        const int nchunks = jb + 1;                      // rows 0 .. 64 (jb + 1) - 1
        int nxt[B];
        fetch_labels(0, nxt);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();                 // previous block's reads of buffer 0 are done
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        store_labels(0, nxt);
        // Chunks before the last hold rows i < 64 jb <= j (and i < N) only, so their C
        // loads need no test; lanes past N read column N - 1 and are never stored.
        // Those loads go through a buffer descriptor over C: the lane's column offset
        // stays in one register and the row offset is a scalar, so a load costs no
        // vector address arithmetic.
        const int jc = jok ? j : N - 1;
        const uint32_t jc_off = 8u * (uint32_t)jc;
        auto chunk = [&](auto checked_tag, int ch) {
            constexpr bool checked = decltype(checked_tag)::value;
            auto cload = [&](int i) -> double {
                if constexpr (checked) return fp64_c(C, N, i, j);
                else return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(c_r, jc_off, 8u * (uint32_t)i * (uint32_t)N, 0));
            };
            const int i0 = ch * 64;
            const int buf = ch & 1;
            if (ch + 1 < nchunks) fetch_labels(i0 + 64, nxt);   // in flight during this chunk
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

            double cq[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) cq[q] = cload(i0 + q);
            for (int r = 0; r < 64; r += 4) {
                double cur[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) cur[q] = cq[q];
                if (r + 4 < 64) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) cq[q] = cload(i0 + r + 4 + q);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const double c = cur[q];
                    int rl[B];
#pragma unroll
                    for (int u = 0; u < B / 4; ++u) {
                        const int4 v = lab_s[wave][buf][r + q][u];
                        rl[4 * u + 0] = v.x;
                        rl[4 * u + 1] = v.y;
                        rl[4 * u + 2] = v.z;
                        rl[4 * u + 3] = v.w;
                    }
                    if constexpr (B == 16) add_if_equal16(acc, rl, lj, c);
                    else add_if_equal8(acc, rl, lj, c);
                }
            }
            if (ch + 1 < nchunks) store_labels(buf ^ 1, nxt);
        };
        for (int ch = 0; ch + 1 < nchunks; ++ch) chunk(std::false_type{}, ch);
        chunk(std::true_type{}, nchunks - 1);
        if (jok) {
            const double cjj = gld(C + (size_t)j * N + j);
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int p = pbase + b;
                if (p < P) gst(d.wsum + (size_t)p * N + j, fma(2.0, acc[b], cjj));
            }
        }
    }
}

hipError_t launch_pairsum_fp64(Tables t, int total_tiles, int parity, const Variant &v, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    if (v.ipg == 16)
        hipLaunchKernelGGL(k_pairsum_fp64<16>, dim3(total_tiles), dim3(256), 0, s, t, parity, v.order);
    else if (v.ipg == 8)
        hipLaunchKernelGGL(k_pairsum_fp64<8>, dim3(total_tiles), dim3(256), 0, s, t, parity, v.order);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Finish: one 256-thread workgroup per individual.
//   1. validity of labels and of v_j; max |v_j| (order-free);
//   2. n_s and sum_{j in s} v_j by integer LDS atomics, v_j scaled by 2^sc and
//      rounded to int64 (sc chosen per individual so N max|v| 2^sc < 2^62:
//      the integer sums are exact and order-free, error <= n_s 2^-(sc+1));
//   3. per label s with n_s > 1: c_s, domain check, the two FP64 log terms
//      of Eq. 8 in literal form. Wave w lists the labels of the w-th quarter
//      of [0, N) with n_s > 1 in ascending order (ballot + prefix); thread t
//      takes entries t, t + 256, ... of the four lists in wave order and sums
//      their terms in that order, each wave adds its lanes by a butterfly, and
//      the four wave sums are added in wave order (a fixed order).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v = fmax(v, __shfl_xor(v, m, 64));
    return v;
}

constexpr int kFinWaves = 4;
constexpr int kFinThreads = 64 * kFinWaves;
constexpr int kFinCache = 8;                       // stocks per thread kept in registers (N <= 2048)

// LDS of the finish workgroup: csum (int64) [N], cnt (int32) [N], the label
// lists (uint16, a quarter of N per wave), then per-wave reduction slots.
// Arrays are padded to 16 bytes (64-bit LDS atomics need aligned addresses).
__host__ __device__ constexpr size_t finish_csum_bytes(int max_n) {
    return ((size_t)max_n * sizeof(long long) + 15) / 16 * 16;
}
__host__ __device__ constexpr size_t finish_cnt_bytes(int max_n) {
    return ((size_t)max_n * sizeof(int) + 15) / 16 * 16;
}
__host__ __device__ constexpr int finish_quarter(int max_n) {
    return (max_n + kFinWaves - 1) / kFinWaves;
}
__host__ __device__ constexpr size_t finish_lst_bytes(int max_n) {
    return ((size_t)kFinWaves * finish_quarter(max_n) * sizeof(uint16_t) + 15) / 16 * 16;
}
__host__ __device__ constexpr size_t finish_lds_bytes(int max_n) {
    // 14.1 KB at N = 1024 (eight workgroups per CU), 57 KB at N = 4096
    return finish_csum_bytes(max_n) + finish_cnt_bytes(max_n) + finish_lst_bytes(max_n) +
           2 * kFinWaves * sizeof(double) + kFinWaves * sizeof(int);
}
// Every region of the layout starts 16-byte aligned for every N the library takes (a 64-bit LDS
// atomic at a misaligned address through a generic pointer faults), and the whole fits in LDS.
constexpr bool finish_layout_ok() {
    for (int n = 1; n <= PGA_N_MAX; ++n) {
        if (finish_csum_bytes(n) % 16 || finish_cnt_bytes(n) % 16 || finish_lst_bytes(n) % 16) return false;
        if (finish_lds_bytes(n) > (size_t)kMaxLdsBytes) return false;
    }
    return true;
}
static_assert(finish_layout_ok(), "finish LDS layout: aligned regions within the LDS limit");

// Per-label outputs and the log terms of Eq. 8 from n_s (cnt) and c_s held in
// 64-bit fixed point (csum, scale 2^sc); thread 0 writes fitness[p]. Called by
// all threads of a kFinThreads workgroup after the barrier that closed the
// writes to cnt and csum. lst holds kFinWaves lists of lst_stride labels;
// nlw holds kFinWaves ints.
__device__ __forceinline__ void finish_terms(const InstDesc &d, int p, int N, const int *cnt,
                                             const long long *csum, int sc, uint16_t *lst, int lst_stride,
                                             double *red, int *nlw, int32_t *status) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    // Pass A (wave w, labels [w Q, (w + 1) Q)): per-label outputs, and the labels
    // with n_s > 1 compacted in ascending order; the four lists, in wave order,
    // list every such label of the individual in ascending order.
    const int QN = finish_quarter(N);                // this instance's quarter; storage is sized by max_n
    const int s_lo = wave * QN, s_hi = min(N, s_lo + QN);
    uint16_t *wl = lst + (size_t)wave * lst_stride;
    int nlist = 0;
    for (int s0 = s_lo; s0 < s_hi; s0 += 64) {
        const int s = s0 + lane;
        const int n = s < s_hi ? cnt[s] : 0;
        if (s < s_hi) {
            if (d.n_s_out) gst(d.n_s_out + (size_t)p * N + s, n);
            if (d.c_s_out) gst(d.c_s_out + (size_t)p * N + s, ldexp((double)csum[s], -sc));
        }
        const uint64_t m = __ballot(n > 1);
        if (n > 1) wl[nlist + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)s;
        nlist += __popcll(m);
    }
    if (lane == 0) nlw[wave] = nlist;
    __syncthreads();

    // Pass B: the two FP64 log terms of Eq. 8 for each listed cluster; entry m of
    // the concatenated lists goes to thread m mod 256, so the (FP64, costly) terms
    // are spread over the whole workgroup rather than over one wave per quarter.
    int pre[kFinWaves + 1];
    pre[0] = 0;
#pragma unroll
    for (int w = 0; w < kFinWaves; ++w) pre[w + 1] = pre[w] + nlw[w];
    double L = 0.0;
    int nbad = 0;
    for (int m = tid; m < pre[kFinWaves]; m += kFinThreads) {
        int w = 0;
#pragma unroll
        for (int v = 1; v < kFinWaves; ++v) w += m >= pre[v] ? 1 : 0;
        const int s = lst[(size_t)w * lst_stride + (m - pre[w])];
        const double nd = (double)cnt[s];
        const double c = ldexp((double)csum[s], -sc);
        const double n2 = nd * nd;
        if (!(c > 0.0 && c < n2)) {
            nbad += 1;
        } else {
            L += log(nd / c) + (nd - 1.0) * log((n2 - nd) / (n2 - c));
        }
    }
    {
        const double wl_sum = wave_sum(L);
        const double wb_sum = wave_sum((double)nbad);
        if (lane == 0) {
            red[wave] = wl_sum;                      // every read of red above precedes the
            red[kFinWaves + wave] = wb_sum;          // barrier that closed the atomics
        }
    }
    __syncthreads();
    if (tid == 0) {
        double Ltot = 0.0, badtot = 0.0;
        for (int w = 0; w < kFinWaves; ++w) {
            Ltot += red[w];
            badtot += red[kFinWaves + w];
        }
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

// The finish of individual p of instance k by one kFinThreads workgroup (every
// thread; the early returns are uniform over the workgroup).
__device__ __forceinline__ void finish_one(const Tables &t, int k, int p, int max_n, int parity, int32_t *status,
                                           unsigned char *smem) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;                     // uniform over the workgroup
    const int N = d.N;
    if (d.route && gld(d.route + p) == 0) return;    // evaluated by the cluster-pair kernel
    const int32_t *__restrict__ lab = d.pop[parity] + (size_t)p * N;
    const double *__restrict__ v = d.wsum + (size_t)p * N;
    long long *csum = (long long *)smem;
    int *cnt = (int *)(smem + finish_csum_bytes(max_n));
    uint16_t *lst = (uint16_t *)(smem + finish_csum_bytes(max_n) + finish_cnt_bytes(max_n));
    double *red = (double *)(smem + finish_csum_bytes(max_n) + finish_cnt_bytes(max_n) + finish_lst_bytes(max_n));

    // Stocks j = tid + 256 u; the first kFinCache per thread stay in registers (all
    // loads issued together), later ones are read again in the accumulation pass.
    // ucache: cached slots in use, uniform over the workgroup, so the slots past N
    // cost nothing (not even masked-off instructions).
    const int ucache = min(kFinCache, (N + kFinThreads - 1) / kFinThreads);
    int lr[kFinCache];
    double vr[kFinCache];
#pragma unroll
    for (int u = 0; u < kFinCache; ++u) {
        if (u >= ucache) break;
        const int j = tid + kFinThreads * u;
        lr[u] = j < N ? gld(lab + j) : 0;
        vr[u] = j < N ? gld(v + j) : 0.0;
    }
    int bad = 0;
    double mx = 0.0;
#pragma unroll
    for (int u = 0; u < kFinCache; ++u) {
        if (u >= ucache) break;
        if (lr[u] < 0 || lr[u] >= N) bad |= 1;
        if (!isfinite(vr[u])) bad |= 2;
        else mx = fmax(mx, fabs(vr[u]));
    }
    for (int j = tid + kFinThreads * kFinCache; j < N; j += kFinThreads) {
        const int l = gld(lab + j);
        if (l < 0 || l >= N) bad |= 1;
        const double x = gld(v + j);
        if (!isfinite(x)) bad |= 2;
        else mx = fmax(mx, fabs(x));
    }
    for (int s = tid; s < N; s += kFinThreads) {
        csum[s] = 0;
        cnt[s] = 0;
    }
    {
        const double wmx = wave_max(mx);
        const double wbad = (double)((__any(bad & 1) ? 1 : 0) | (__any(bad & 2) ? 2 : 0));
        if (lane == 0) {
            red[wave] = wmx;
            red[kFinWaves + wave] = wbad;
        }
    }
    __syncthreads();
    int any_bad = 0;
#pragma unroll
    for (int w = 0; w < kFinWaves; ++w) {
        mx = fmax(mx, red[w]);
        any_bad |= (int)red[kFinWaves + w];
    }
    if (any_bad) {
        if (tid == 0) {
            d.fitness[p] = -INFINITY;
            if (status) {
                if (any_bad & 1) atomicAdd(&status[PGA_ST_LABEL], 1);
                atomicAdd(&status[PGA_ST_NONFINITE], 1);
            }
        }
        if (d.n_s_out)
            for (int s = tid; s < N; s += kFinThreads) d.n_s_out[(size_t)p * N + s] = 0;
        if (d.c_s_out)
            for (int s = tid; s < N; s += kFinThreads) d.c_s_out[(size_t)p * N + s] = 0.0;
        return;                                      // uniform: any_bad is the same for every thread
    }
    int sc = 0;
    if (mx > 0.0) {
        int e;
        frexp(mx * (double)N, &e);                   // N max|v| < 2^e
        sc = 61 - e;
    }
#pragma unroll
    for (int u = 0; u < kFinCache; ++u) {
        if (u >= ucache) break;
        if (tid + kFinThreads * u < N) {
            atomicAdd(&cnt[lr[u]], 1);
            atomicAdd((unsigned long long *)&csum[lr[u]], (unsigned long long)llrint(ldexp(vr[u], sc)));
        }
    }
    for (int j = tid + kFinThreads * kFinCache; j < N; j += kFinThreads) {
        const int l = gld(lab + j);
        const long long q = llrint(ldexp(gld(v + j), sc));
        atomicAdd(&cnt[l], 1);
        atomicAdd((unsigned long long *)&csum[l], (unsigned long long)q);
    }
    __syncthreads();

    finish_terms(d, p, N, cnt, csum, sc, lst, finish_quarter(max_n), red, (int *)(red + 2 * kFinWaves), status);
}

// Workgroup g takes individual g.
__global__ __launch_bounds__(kFinThreads) void k_finish(Tables t, int max_n, int parity, int32_t *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int g = blockIdx.x;
    if (g >= t.inds[t.n_inst]) return;               // the grid may exceed the total (capacity-sized graph)
    const int k = find_inst(t.inds, t.n_inst, g);
    finish_one(t, k, g - t.inds[k], max_n, parity, status, smem);
}

// Listed (cluster-pair route on, large launches): per slice of this parity's
// dense list, `per` workgroups (gridDim.x = slices * per) take its entries at,
// at + per, ... below the slice's length, so a list that is nearly empty costs a
// small launch rather than a workgroup per possible entry. (A kernel of its own:
// the loop needs more registers than the one-individual form.)
__global__ __launch_bounds__(kFinThreads) void k_finish_listed(Tables t, int max_n, int parity, int slices, int cap,
                                                               int32_t *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int slice = (int)blockIdx.x % slices, per = (int)gridDim.x / slices;
    const int n = __builtin_amdgcn_readfirstlane(gld(list_count(t, parity, kListDense, slice)));
    for (int at = (int)blockIdx.x / slices; at < n; at += per) {
        const int32_t *e = list_entry(t, kListDense, slice, cap, at);
        const int p = __builtin_amdgcn_readfirstlane(gld(e));
        const int k = __builtin_amdgcn_readfirstlane(gld(e + 1));
        finish_one(t, k, p, max_n, parity, status, smem);
        __syncthreads();                             // the next entry reuses the LDS
    }
}

// Workgroups per dense-list slice in a listed finish (at most the slice capacity).
constexpr int kFinListPerSlice = 8;

hipError_t launch_finish(Tables t, int total_inds, int max_n, int parity, int listed, int32_t *status,
                         hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    const int n_wg = (total_inds + 3) / 4, slices = list_slices(n_wg), cap = list_slice_cap(n_wg);
    const int per = cap < kFinListPerSlice ? cap : kFinListPerSlice;
    if (listed)
        hipLaunchKernelGGL(k_finish_listed, dim3(slices * per), dim3(kFinThreads), finish_lds_bytes(max_n), s, t, max_n,
                           parity, slices, cap, status);
    else
        hipLaunchKernelGGL(k_finish, dim3(total_inds), dim3(kFinThreads), finish_lds_bytes(max_n), s, t, max_n, parity,
                           status);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cluster-pair fitness (exact FP64 route). c_s of Eq. 6 only involves the pairs
// inside cluster s, so an individual with few such pairs is evaluated from
// them directly instead of by the O(N^2) pair-sum: one 256-thread workgroup
// per individual
//   1. labels and the diagonal of C (a contiguous copy; not read when every
//      C_jj is 1) into registers, the labels also into LDS (invalid labels:
//      fitness -inf, as the finish does);
//   2. n_s by LDS atomics; pairs = sum_s n_s (n_s - 1) / 2 and max n_s;
//   3. pairs above the limit: route[p] = 1 (the pair-sum and finish kernels
//      evaluate it) and stop;
//   4. members grouped by cluster (counting sort on the exclusive prefix of
//      n_s); the same scan gives PP, the exclusive prefix of the pair counts
//      n_s (n_s - 1) / 2, which numbers the pairs: pair q belongs to the
//      cluster s with PP[s] <= q < PP[s+1], and r = q - PP[s] = b (b-1)/2 + a
//      (a < b) joins its members a and b;
//   5. c_s = sum_{j in s} C_jj + 2 sum_{pairs} C_ij (upper triangle, as the
//      FP64 pair-sum reads it) accumulated in 64-bit fixed point: with
//      |C| <= 1 every partial sum is bounded by max n_s^2, and the scale 2^sc
//      keeps max n_s^2 2^sc <= 2^61, so the integer sums are exact and the
//      result does not depend on the order of the atomics;
//   6. an entry with |C| > 1 or not finite sends the individual to the dense
//      route (step 3's flag), which treats it exactly as before; otherwise
//      route[p] = 0 and the log terms follow as in the finish.
constexpr int kSparseMaxN = 2048;                  // larger instances always take the dense route
constexpr int kSparseCache = kSparseMaxN / kFinThreads;   // stocks per thread, all in registers

__host__ __device__ constexpr size_t pad16(size_t b) { return (b + 15) / 16 * 16; }
__host__ __device__ constexpr size_t sparse_members_bytes(int n) {
    const size_t m = pad16(2 * (size_t)n), l = finish_lst_bytes(n);
    return m > l ? m : l;
}
// LDS: csum int64[n] | cnt int32[n] | begin int32[n + 1] | PP int32[n + 1] | members,
// then the finish lists | kFinWaves x 2 doubles | 16 int32.
// 22.7 KB at N = 1024 (seven workgroups per CU).
__host__ __device__ constexpr size_t sparse_lds_bytes(int n) {
    return pad16(8 * (size_t)n) + pad16(4 * (size_t)n) + 2 * pad16(4 * ((size_t)n + 1)) + sparse_members_bytes(n) +
           2 * kFinWaves * sizeof(double) + 16 * sizeof(int);
}
constexpr bool sparse_layout_ok() {
    for (int n = 1; n <= kSparseMaxN; ++n) {
        if (sparse_members_bytes(n) % 16) return false;
        if (sparse_lds_bytes(n) > (size_t)kMaxLdsBytes) return false;
    }
    return true;
}
static_assert(sparse_layout_ok(), "cluster-pair LDS layout: aligned regions within the LDS limit");

// Exclusive prefixes of n_s (begin) and of n_s (n_s - 1) / 2 (pp) over
// [0, n), as block_exscan; returns the number of pairs and sets nmax to the
// largest n_s; wtot: 12 ints.
__device__ __forceinline__ int block_exscan_cnt_pairs(const int *cnt, int *begin, int *pp, int n, int *wtot,
                                                      int &nmax) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + kFinThreads - 1) / kFinThreads;
    const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
    int own = 0, ownp = 0, mx = 0;
    for (int x = b0; x < b1; ++x) {
        const int c = cnt[x];
        own += c;
        ownp += c * (c - 1) / 2;
        mx = max(mx, c);
    }
    int inc = own, incp = ownp;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64), yp = __shfl_up(incp, o, 64);
        if (lane >= o) {
            inc += y;
            incp += yp;
        }
        mx = max(mx, __shfl_xor(mx, o, 64));
    }
    if (lane == 63) {
        wtot[wave] = inc;
        wtot[kFinWaves + wave] = incp;
        wtot[2 * kFinWaves + wave] = mx;
    }
    __syncthreads();
    int run = inc - own, runp = incp - ownp, totalp = 0;
    nmax = 0;
#pragma unroll
    for (int w = 0; w < kFinWaves; ++w) {
        if (w < wave) {
            run += wtot[w];
            runp += wtot[kFinWaves + w];
        }
        totalp += wtot[kFinWaves + w];
        nmax = max(nmax, wtot[2 * kFinWaves + w]);
    }
    for (int x = b0; x < b1; ++x) {
        const int c = cnt[x];
        begin[x] = run;
        pp[x] = runp;
        run += c;
        runp += c * (c - 1) / 2;
    }
    __syncthreads();
    return totalp;
}

// Exclusive prefix sum of a[0 .. n) into out (may alias a); thread t scans a
// contiguous run of ceil(n / 256). Returns the total; ends with a barrier.
__device__ __forceinline__ int block_exscan(const int *a, int *out, int n, int *wtot) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int per = (n + kFinThreads - 1) / kFinThreads;
    const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
    int own = 0;
    for (int x = b0; x < b1; ++x) own += a[x];
    int inc = own;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
    }
    if (lane == 63) wtot[wave] = inc;
    __syncthreads();
    int run = inc - own, total = 0;
#pragma unroll
    for (int w = 0; w < kFinWaves; ++w) {
        if (w < wave) run += wtot[w];
        total += wtot[w];
    }
    for (int x = b0; x < b1; ++x) {
        const int v = a[x];
        out[x] = run;
        run += v;
    }
    __syncthreads();
    return total;
}

__device__ __forceinline__ unsigned long long fixed_pt(double c, int sc) {
    return (unsigned long long)llrint(ldexp(c, sc));
}

// Route of every individual, one wave each (four per workgroup): n_s by LDS
// atomics, whose return values add up to the pair count sum_s n_s (n_s - 1) / 2
// exactly. An individual at or under the limit, or with a label outside
// [0, N), goes to the sparse list (route 0), the others to the dense list
// (route 1). Workgroup w appends to slice w mod slices of each list with
// one atomic per list; the order within a slice depends on timing, the
// content does not. Workgroup 0 also empties the other parity's lists.
__global__ __launch_bounds__(256) void k_route(Tables t, int lds_n, int parity, double frac, int slices, int cap) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int kind[4], ent[4][2];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (blockIdx.x == 0)
        for (int i = threadIdx.x; i < 2 * kListSlices; i += 256) gst(t.sq + (2 * (parity ^ 1)) * kListSlices + i, 0);
    const int g = __builtin_amdgcn_readfirstlane(4 * (int)blockIdx.x + wave);
    int mine = -1, k = 0, p = 0;                     // mine: the list this wave's individual joins
    if (g < t.inds[t.n_inst]) {                      // the grid may exceed the total (capacity-sized graph)
        k = find_inst(t.inds, t.n_inst, g);
        const InstDesc &d = t.desc[k];
        const int N = d.N;
        p = g - t.inds[k];
        if (inst_stopped(d)) {
        } else if (N > lds_n) {                      // lds_n <= kSparseMaxN
            if (lane == 0) gst(d.route + p, 1);
            mine = kListDense;
        } else if (N <= kRouteAllPairsMaxN) {        // within the limit whatever its labels
            if (lane == 0) gst(d.route + p, 0);
            mine = kListSparse;
        } else {
            int *cnt = (int *)(smem + (size_t)wave * pad16(4 * (size_t)lds_n));
            for (int s = lane; s < N; s += 64) cnt[s] = 0;
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            const int32_t *__restrict__ lab = d.pop[parity] + (size_t)p * N;
            int pairs = 0, bad = 0;
            for (int j0 = lane; j0 < N; j0 += 4 * 64) {     // four labels per lane in flight
                int l[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) l[u] = j0 + 64 * u < N ? gld(lab + j0 + 64 * u) : 0;
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (j0 + 64 * u >= N) break;
                    if (l[u] < 0 || l[u] >= N) bad = 1;
                    else pairs += atomicAdd(&cnt[l[u]], 1);
                }
            }
#pragma unroll
            for (int m = 32; m > 0; m >>= 1) pairs += __shfl_xor(pairs, m, 64);
            const bool sparse = __any(bad) || (double)pairs <= route_limit(N, frac);
            if (lane == 0) gst(d.route + p, sparse ? 0 : 1);
            mine = sparse ? kListSparse : kListDense;
        }
    }
    if (lane == 0) {
        kind[wave] = mine;
        ent[wave][0] = p;
        ent[wave][1] = k;
    }
    __syncthreads();
    if (threadIdx.x < 2) {                           // thread L appends this workgroup's individuals of list L
        const int L = threadIdx.x;
        int n = 0;
#pragma unroll
        for (int w = 0; w < 4; ++w) n += kind[w] == L ? 1 : 0;
        if (n > 0) {
            const int slice = (int)blockIdx.x % slices;
            int at = atomicAdd(list_count(t, parity, L, slice), n);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (kind[w] == L) {
                    int32_t *e = list_entry(t, L, slice, cap, at++);
                    gst(e, ent[w][0]);
                    gst(e + 1, ent[w][1]);
                }
        }
    }
}

// An individual the cluster-pair kernel hands back to the pair-sum route joins
// the dense list (one thread; the slice it came from has room for it there).
// slice < 0: no lists in use (the finish reads every individual's route).
__device__ __forceinline__ void list_dense(const Tables &t, int parity, int slice, int cap, int p, int k) {
    if (slice < 0) return;
    int32_t *e = list_entry(t, kListDense, slice, cap, atomicAdd(list_count(t, parity, kListDense, slice), 1));
    gst(e, p);
    gst(e + 1, k);
}

__host__ __device__ constexpr size_t route_lds_bytes(int n) { return 4 * pad16(4 * (size_t)n); }
static_assert(route_lds_bytes(kSparseMaxN) <= (size_t)kMaxLdsBytes, "route LDS within the limit");

// The cluster-pair evaluation of individual p of instance k (all threads of the
// workgroup), taken from slice `slice` of the sparse list. An individual it
// hands to the pair-sum route (route 1) joins the dense list.
__device__ void sparse_one(const Tables &t, int k, int p, int slice, int cap, int lds_n, int parity, double frac,
                           int32_t *status, unsigned char *smem) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, tid = threadIdx.x;
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;                     // uniform over the workgroup
    const int N = d.N;
    if (N > lds_n) {                                 // lds_n <= kSparseMaxN
        if (tid == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;
    }
    const size_t n = (size_t)lds_n;
    unsigned char *b = smem;
    long long *csum = (long long *)b;   b += pad16(8 * n);
    int *cnt = (int *)b;                b += pad16(4 * n);
    int *begin = (int *)b;              b += pad16(4 * (n + 1));
    int *PP = (int *)b;                 b += pad16(4 * (n + 1));
    uint16_t *members = (uint16_t *)b;  b += sparse_members_bytes(lds_n);
    uint16_t *lst = members;            // the finish lists replace members after the pairs
    double *red = (double *)b;          b += 2 * kFinWaves * sizeof(double);
    int *ired = (int *)b;               // [0, 4) flags, [4, 16) scan totals, then [12, 16) list lengths

    const int32_t *__restrict__ lab = d.pop[parity] + (size_t)p * N;
    const double *__restrict__ C = d.C;

    // Stocks j = tid + 256 u, u < ucache (uniform), all of them (N <= 2048).
    const int ucache = (N + kFinThreads - 1) / kFinThreads;
    const bool ones = gld(d.diag + N) == 1.0;        // every C_jj is 1 (uniform)
    int lr[kSparseCache];
    double dg[kSparseCache];
#pragma unroll
    for (int u = 0; u < kSparseCache; ++u) {
        if (u >= ucache) break;
        const int j = tid + kFinThreads * u;
        lr[u] = j < N ? gld(lab + j) : 0;
        dg[u] = (!ones && j < N) ? gld(d.diag + j) : 1.0;
    }
    int bad = 0;
#pragma unroll
    for (int u = 0; u < kSparseCache; ++u) {
        if (u >= ucache) break;
        const int j = tid + kFinThreads * u;
        if (j < N) {
            if (lr[u] < 0 || lr[u] >= N) bad = 1;
            cnt[j] = 0;
            csum[j] = 0;
        }
    }
    const int wbad = __any(bad) ? 1 : 0;             // all lanes vote, lane 0 records
    if (lane == 0) ired[wave] = wbad;
    __syncthreads();
    if (ired[0] | ired[1] | ired[2] | ired[3]) {     // as the finish: labels outside [0, N)
        if (tid == 0) {
            gst(d.route + p, 0);
            d.fitness[p] = -INFINITY;
            if (status) {
                atomicAdd(&status[PGA_ST_LABEL], 1);
                atomicAdd(&status[PGA_ST_NONFINITE], 1);
            }
        }
        if (d.n_s_out)
            for (int s = tid; s < N; s += kFinThreads) d.n_s_out[(size_t)p * N + s] = 0;
        if (d.c_s_out)
            for (int s = tid; s < N; s += kFinThreads) d.c_s_out[(size_t)p * N + s] = 0.0;
        return;
    }
#pragma unroll
    for (int u = 0; u < kSparseCache; ++u) {
        if (u >= ucache) break;
        if (tid + kFinThreads * u < N) atomicAdd(&cnt[lr[u]], 1);
    }
    __syncthreads();

    // begin[s]: first position of cluster s; PP[s]: pairs of the clusters below s
    int nmax;
    const int T = block_exscan_cnt_pairs(cnt, begin, PP, N, ired + 4, nmax);   // T == pairs
    if ((double)T > route_limit(N, frac)) {
        if (tid == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;                                      // uniform
    }
    int e;
    frexp((double)nmax * (double)nmax, &e);          // max n_s^2 < 2^e
    const int sc = 61 - e;
    if (tid == 0) PP[N] = T;
    int badc = 0;
#pragma unroll
    for (int u = 0; u < kSparseCache; ++u) {
        if (u >= ucache) break;
        const int j = tid + kFinThreads * u;
        if (j < N) {
            members[atomicAdd(&begin[lr[u]], 1)] = (uint16_t)j;
            if (!ones) {
                if (!(fabs(dg[u]) <= 1.0)) badc = 1;
                else atomicAdd((unsigned long long *)&csum[lr[u]], fixed_pt(dg[u], sc));
            }
        }
    }
    if (ones)                                        // sum of n_s diagonal ones, exact
        for (int s = tid; s < N; s += kFinThreads) csum[s] = (long long)cnt[s] << sc;
    __syncthreads();                                 // begin[s] is now the end of cluster s

    // Each thread takes kq consecutive pairs per round (one search, then a forward
    // walk) with their loads issued together; kq = ceil(T / 256), at most kQ, so
    // every thread has work. Consecutive pairs mostly share a cluster, so the
    // terms are summed in a register while the label stays the same and added to
    // csum once per run (fewer atomics on one LDS address).
    constexpr int kQ = 8;
    const int kq = min(kQ, max(1, (T + kFinThreads - 1) / kFinThreads));   // uniform
    for (int q0 = tid * kq; q0 < T; q0 += kq * kFinThreads) {
        int cs = 0, hi = N;                          // PP[cs] <= q0 < PP[hi]
        while (hi - cs > 1) {
            const int mid = (cs + hi) >> 1;
            if (PP[mid] <= q0) cs = mid;
            else hi = mid;
        }
        const int r = q0 - PP[cs];                   // = bq (bq - 1) / 2 + aq, aq < bq
        int bq = (int)((1.0 + sqrt(1.0 + 8.0 * (double)r)) * 0.5);
        while (bq * (bq - 1) / 2 > r) --bq;
        while ((bq + 1) * bq / 2 <= r) ++bq;
        int aq = r - bq * (bq - 1) / 2;
        int st = begin[cs] - cnt[cs];                // first position of cluster cs
        int pend = PP[cs + 1];                       // first pair of the clusters above cs
        double c[kQ];
        int l[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const int q = q0 + u;
            l[u] = -1;
            c[u] = 0.0;
            if (u < kq && q < T) {
                while (q >= pend) {                  // next cluster with pairs (PP[N] = T > q)
                    ++cs;
                    pend = PP[cs + 1];
                    st = begin[cs] - cnt[cs];
                    aq = 0;
                    bq = 1;
                }
                const int j = members[st + bq], i = members[st + aq];
                c[u] = gld(C + (size_t)min(i, j) * N + max(i, j));
                l[u] = cs;
                if (++aq == bq) {
                    ++bq;
                    aq = 0;
                }
            }
        }
        long long run = 0;
        int cur = -1;
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            if (l[u] < 0) continue;
            if (!(fabs(c[u]) <= 1.0)) {
                badc = 1;
                continue;
            }
            if (l[u] != cur) {
                if (cur >= 0) atomicAdd((unsigned long long *)&csum[cur], (unsigned long long)run);
                cur = l[u];
                run = 0;
            }
            run += fixed_pt(2.0 * c[u], sc);
        }
        if (cur >= 0) atomicAdd((unsigned long long *)&csum[cur], (unsigned long long)run);
    }
    const int wbadc = __any(badc) ? 1 : 0;
    if (lane == 0) ired[wave] = wbadc;
    __syncthreads();
    if (ired[0] | ired[1] | ired[2] | ired[3]) {
        if (tid == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;
    }
    if (tid == 0) gst(d.route + p, 0);
    finish_terms(d, p, N, cnt, csum, sc, lst, finish_quarter(lds_n), red, ired + 12, status);
}

// The same evaluation by one wave (a 64-thread workgroup) for N <= 512: at the
// batched form's sizes a whole workgroup per individual repeats its scans,
// reductions and barriers in every wave and holds eight individuals per
// compute unit. The steps and their integer results are those of sparse_one;
// the log terms are added in the workgroup kernel's order (entry m of the
// label list to virtual thread m mod 256, each virtual wave's lanes by the
// same butterfly, the four virtual waves in order), so the fitness has the
// same bits whichever of the two kernels evaluates it.
// LDS (18 N bytes): csum int64 [N] | n_s, then the cluster starts, then their
// ends, int32 [N + 1] | PP int32 [N + 1] | members uint16 [N], later the list
// of labels with n_s > 1.
constexpr int kSparseWaveMaxN = 512;
constexpr int kSwCache = kSparseWaveMaxN / 64;     // stocks per lane, all in registers

__host__ __device__ constexpr size_t sparse_wave_lds_bytes(int n) {
    return pad16(8 * (size_t)n) + 2 * pad16(4 * ((size_t)n + 1)) + pad16(2 * (size_t)n);
}
static_assert(sparse_wave_lds_bytes(kSparseWaveMaxN) <= (size_t)kMaxLdsBytes, "wave cluster-pair LDS");

// Orders the LDS accesses of the wave's lanes (one wave: no barrier needed).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ void sparse_one_wave(const Tables &t, int k, int p, int slice, int cap, int lds_n, int parity,
                                double frac, int32_t *status, unsigned char *smem) {
    const int lane = threadIdx.x;
    const InstDesc &d = t.desc[k];
    if (inst_stopped(d)) return;
    const int N = d.N;
    if (N > lds_n) {                                 // lds_n <= kSparseWaveMaxN
        if (lane == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;
    }
    const size_t n = (size_t)lds_n;
    unsigned char *b = smem;
    long long *csum = (long long *)b;   b += pad16(8 * n);
    int *cb = (int *)b;                 b += pad16(4 * (n + 1));
    int *PP = (int *)b;                 b += pad16(4 * (n + 1));
    uint16_t *members = (uint16_t *)b;
    const int32_t *__restrict__ lab = d.pop[parity] + (size_t)p * N;
    const double *__restrict__ C = d.C;

    const int ucache = (N + 63) / 64;                // uniform
    int lr[kSwCache];
    double dg[kSwCache];
#pragma unroll
    for (int u = 0; u < kSwCache; ++u) {             // the labels are requested first, then the flag
        if (u >= ucache) break;
        const int j = lane + 64 * u;
        lr[u] = j < N ? gld(lab + j) : 0;
    }
    const bool ones = gld(d.diag + N) == 1.0;
#pragma unroll
    for (int u = 0; u < kSwCache; ++u) {
        if (u >= ucache) break;
        const int j = lane + 64 * u;
        dg[u] = (!ones && j < N) ? gld(d.diag + j) : 1.0;
    }
    int bad = 0;
#pragma unroll
    for (int u = 0; u < kSwCache; ++u) {
        if (u >= ucache) break;
        const int j = lane + 64 * u;
        if (j < N) {
            if (lr[u] < 0 || lr[u] >= N) bad = 1;
            cb[j] = 0;
            csum[j] = 0;
        }
    }
    if (__any(bad)) {                                // as the finish: labels outside [0, N)
        if (lane == 0) {
            gst(d.route + p, 0);
            d.fitness[p] = -INFINITY;
            if (status) {
                atomicAdd(&status[PGA_ST_LABEL], 1);
                atomicAdd(&status[PGA_ST_NONFINITE], 1);
            }
        }
        if (d.n_s_out)
            for (int s = lane; s < N; s += 64) d.n_s_out[(size_t)p * N + s] = 0;
        if (d.c_s_out)
            for (int s = lane; s < N; s += 64) d.c_s_out[(size_t)p * N + s] = 0.0;
        return;
    }
    wave_lds_sync();
    // n_s; the atomics' old values add up to the pair count, their maximum + 1 is max n_s
    int T = 0, nmax = 0;
#pragma unroll
    for (int u = 0; u < kSwCache; ++u) {
        if (u >= ucache) break;
        if (lane + 64 * u < N) {
            const int old = atomicAdd(&cb[lr[u]], 1);
            T += old;
            nmax = max(nmax, old + 1);
        }
    }
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        T += __shfl_xor(T, m, 64);
        nmax = max(nmax, __shfl_xor(nmax, m, 64));
    }
    if ((double)T > route_limit(N, frac)) {
        if (lane == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;
    }
    int e;
    frexp((double)nmax * (double)nmax, &e);          // max n_s^2 < 2^e
    const int sc = 61 - e;
    wave_lds_sync();
    // exclusive prefixes of n_s (in place: cluster starts) and of the pair counts
    {
        const int per = (N + 63) / 64;
        const int b0 = min(N, lane * per), b1 = min(N, b0 + per);
        int own = 0, ownp = 0;
        for (int x = b0; x < b1; ++x) {
            const int c = cb[x];
            own += c;
            ownp += c * (c - 1) / 2;
        }
        int inc = own, incp = ownp;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(inc, o, 64), yp = __shfl_up(incp, o, 64);
            if (lane >= o) {
                inc += y;
                incp += yp;
            }
        }
        int run = inc - own, runp = incp - ownp;
        for (int x = b0; x < b1; ++x) {
            const int c = cb[x];
            cb[x] = run;
            PP[x] = runp;
            run += c;
            runp += c * (c - 1) / 2;
        }
        if (lane == 0) PP[N] = T;
    }
    wave_lds_sync();
    // members grouped by cluster; cb[s] becomes the end of cluster s, whose start is cb[s - 1]
    int badc = 0;
#pragma unroll
    for (int u = 0; u < kSwCache; ++u) {
        if (u >= ucache) break;
        const int j = lane + 64 * u;
        if (j < N) {
            members[atomicAdd(&cb[lr[u]], 1)] = (uint16_t)j;
            if (!ones) {
                if (!(fabs(dg[u]) <= 1.0)) badc = 1;
                else atomicAdd((unsigned long long *)&csum[lr[u]], fixed_pt(dg[u], sc));
            }
        }
    }
    wave_lds_sync();
    if (ones)                                        // sum of n_s diagonal ones, exact
        for (int s = lane; s < N; s += 64) csum[s] = (long long)(cb[s] - (s ? cb[s - 1] : 0)) << sc;
    wave_lds_sync();

    // pairs: kq consecutive ones per lane and round, as the workgroup kernel takes them
    constexpr int kQ = 8;
    const int kq = min(kQ, max(1, (T + 63) / 64));   // uniform
    for (int q0 = lane * kq; q0 < T; q0 += kq * 64) {
        int cs = 0, hi = N;                          // PP[cs] <= q0 < PP[hi]
        while (hi - cs > 1) {
            const int mid = (cs + hi) >> 1;
            if (PP[mid] <= q0) cs = mid;
            else hi = mid;
        }
        const int r = q0 - PP[cs];                   // = bq (bq - 1) / 2 + aq, aq < bq
        int bq = (int)((1.0 + sqrt(1.0 + 8.0 * (double)r)) * 0.5);
        while (bq * (bq - 1) / 2 > r) --bq;
        while ((bq + 1) * bq / 2 <= r) ++bq;
        int aq = r - bq * (bq - 1) / 2;
        int st = cs ? cb[cs - 1] : 0;                // first position of cluster cs
        int pend = PP[cs + 1];
        double c[kQ];
        int l[kQ];
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            const int q = q0 + u;
            l[u] = -1;
            c[u] = 0.0;
            if (u < kq && q < T) {
                while (q >= pend) {                  // next cluster with pairs (PP[N] = T > q)
                    st = cb[cs];
                    ++cs;
                    pend = PP[cs + 1];
                    aq = 0;
                    bq = 1;
                }
                const int j = members[st + bq], i = members[st + aq];
                c[u] = gld(C + (size_t)min(i, j) * N + max(i, j));
                l[u] = cs;
                if (++aq == bq) {
                    ++bq;
                    aq = 0;
                }
            }
        }
        long long run = 0;
        int cur = -1;
#pragma unroll
        for (int u = 0; u < kQ; ++u) {
            if (l[u] < 0) continue;
            if (!(fabs(c[u]) <= 1.0)) {
                badc = 1;
                continue;
            }
            if (l[u] != cur) {
                if (cur >= 0) atomicAdd((unsigned long long *)&csum[cur], (unsigned long long)run);
                cur = l[u];
                run = 0;
            }
            run += fixed_pt(2.0 * c[u], sc);
        }
        if (cur >= 0) atomicAdd((unsigned long long *)&csum[cur], (unsigned long long)run);
    }
    if (__any(badc)) {
        if (lane == 0) {
            gst(d.route + p, 1);
            list_dense(t, parity, slice, cap, p, k);
        }
        return;
    }
    if (lane == 0) gst(d.route + p, 0);
    wave_lds_sync();

    // per-label outputs and the list of labels with n_s > 1, ascending (into members)
    uint16_t *lst = members;
    int nlist = 0;
    for (int s0 = 0; s0 < N; s0 += 64) {
        const int s = s0 + lane;
        const int ns = s < N ? cb[s] - (s ? cb[s - 1] : 0) : 0;
        if (s < N) {
            if (d.n_s_out) gst(d.n_s_out + (size_t)p * N + s, ns);
            if (d.c_s_out) gst(d.c_s_out + (size_t)p * N + s, ldexp((double)csum[s], -sc));
        }
        const uint64_t m = __ballot(ns > 1);
        if (ns > 1) lst[nlist + __popcll(m & ((1ull << lane) - 1ull))] = (uint16_t)s;
        nlist += __popcll(m);
    }
    wave_lds_sync();
    // entry m belongs to virtual thread m mod 256, i.e. virtual wave (m / 64) mod 4
    double L[kFinWaves] = {0.0, 0.0, 0.0, 0.0};
    int nbad[kFinWaves] = {0, 0, 0, 0};
    for (int m = lane; m < nlist; m += 64) {
        const int w = (m >> 6) & (kFinWaves - 1);
        const int s = lst[m];
        const int ni = cb[s] - (s ? cb[s - 1] : 0);
        const double nd = (double)ni;
        const double c = ldexp((double)csum[s], -sc);
        const double n2 = nd * nd;
        const bool ok = c > 0.0 && c < n2;
        const double term = ok ? log(nd / c) + (nd - 1.0) * log((n2 - nd) / (n2 - c)) : 0.0;
#pragma unroll
        for (int v = 0; v < kFinWaves; ++v)
            if (v == w) {
                if (ok) L[v] += term;
                else nbad[v] += 1;
            }
    }
    double Ltot = 0.0, badtot = 0.0;
#pragma unroll
    for (int v = 0; v < kFinWaves; ++v) {
        Ltot += wave_sum(L[v]);
        badtot += wave_sum((double)nbad[v]);
    }
    if (lane == 0) {
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

// Listed: entry i / slices of slice i mod slices of this parity's sparse list
// (workgroups past their slice's length end at once). Else individual i, the
// route decided here as in the workgroup kernel.
__device__ __forceinline__ bool sparse_target(const Tables &t, int listed, int parity, int slices, int cap, int &k,
                                              int &p, int &slice) {
    if (listed) {
        slice = (int)blockIdx.x % slices;
        const int at = (int)blockIdx.x / slices;
        const int32_t *e = list_entry(t, kListSparse, slice, cap, at);   // read with the count: in bounds
        const int n = *list_count(t, parity, kListSparse, slice);
        p = __builtin_amdgcn_readfirstlane(gld(e));
        k = __builtin_amdgcn_readfirstlane(gld(e + 1));
        return at < n;
    }
    const int g = blockIdx.x;
    if (g >= t.inds[t.n_inst]) return false;         // the grid may exceed the total (capacity-sized graph)
    k = find_inst(t.inds, t.n_inst, g);
    p = g - t.inds[k];
    slice = -1;
    return true;
}

__global__ __launch_bounds__(64) void k_sparse_wave(Tables t, int lds_n, int parity, double frac, int listed,
                                                    int slices, int cap, int32_t *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    int k, p, slice;
    if (!sparse_target(t, listed, parity, slices, cap, k, p, slice)) return;
    sparse_one_wave(t, k, p, slice, cap, lds_n, parity, frac, status, smem);
}

// A workgroup per list entry or individual (see sparse_target). (A grid-stride
// loop over a smaller grid holds the per-thread values of the body across
// iterations: 85 registers instead of 52, five waves per SIMD instead of
// eight.)
__global__ __launch_bounds__(kFinThreads) void k_sparse(Tables t, int lds_n, int parity, double frac, int listed,
                                                        int slices, int cap, int32_t *status) {
    extern __shared__ __align__(16) unsigned char smem[];
    int k, p, slice;
    if (!sparse_target(t, listed, parity, slices, cap, k, p, slice)) return;
    sparse_one(t, k, p, slice, cap, lds_n, parity, frac, status, smem);
}

hipError_t launch_sparse(Tables t, int total_inds, int max_n, int parity, double frac, int listed, int lists_ready,
                         int32_t *status, hipStream_t s) {
    if (total_inds <= 0) return hipSuccess;
    const int n = std::min(max_n, kSparseMaxN);
    const int n_wg = (total_inds + 3) / 4, slices = list_slices(n_wg), cap = list_slice_cap(n_wg);
    if (listed && !lists_ready) {
        hipLaunchKernelGGL(k_route, dim3(n_wg), dim3(256), route_lds_bytes(n), s, t, n, parity, frac, slices, cap);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int grid = listed ? slices * cap : total_inds;
    if (n <= kSparseWaveMaxN)
        hipLaunchKernelGGL(k_sparse_wave, dim3(grid), dim3(64), sparse_wave_lds_bytes(n), s, t, n, parity, frac,
                           listed, slices, cap, status);
    else
        hipLaunchKernelGGL(k_sparse, dim3(grid), dim3(kFinThreads), sparse_lds_bytes(n), s, t, n, parity, frac,
                           listed, slices, cap, status);
    return hipGetLastError();
}

// Contiguous copy of the diagonal of every instance's C (one workgroup per
// instance, blockIdx.y), and diag[N] = 1 if every C_jj is 1, else 0.
__global__ __launch_bounds__(256) void k_diag(Tables t) {
    const InstDesc &d = t.desc[blockIdx.y];
    if (!d.diag || d.P == 0) return;                 // uniform
    int ones = 1;
    for (int j = threadIdx.x; j < d.N; j += 256) {
        const double c = gld(d.C + (size_t)j * d.N + j);
        gst(d.diag + j, c);
        ones &= c == 1.0 ? 1 : 0;
    }
    const int all = __syncthreads_and(ones);
    if (threadIdx.x == 0) gst(d.diag + d.N, all ? 1.0 : 0.0);
}

hipError_t launch_diag(Tables t, int max_n, hipStream_t s) {
    if (t.n_inst <= 0 || max_n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_diag, dim3(1, t.n_inst), dim3(256), 0, s, t);
    return hipGetLastError();
}

}  // namespace pga
