// BF16x2 pair-sum on MFMA: v_pj = C_jj + 2 sum_{i<j} [s_pi = s_pj] (hi_ji + lo_ji),
// the sum over i being the diagonal of a one-hot contraction (c_s is the
// diagonal of Y^T C Y, Eq. 6).
//
// One wave owns 16 stocks j = jt0 .. jt0+15 and walks the rows i < j in
// chunks of 32 with v_mfma_f32_16x16x32_bf16:
//   A[m][k] = C[jt0 + m][i0 + k]           (hi, then lo: two MFMAs)
//   B[k][n] = [s_{i0+k} = s_{jt0+n}] [i0 + k < jt0 + n]   (0 or bf16 1.0)
//   D[m][n] += sum_k A[m][k] B[k][n];  D[n][n] = partial sum for stock jt0+n
// Lane l supplies row m = l%16 of A and column n = l%16 of B over the same
// eight k = 8(l/16)..+7, so its A row and B column are both stock jt0 + l%16:
// the lane needs only its own stock's label and the 8 row labels of its k
// block. The one-hot column costs 3 packed 16-bit ALU ops per 2 rows (xor,
// saturating 1 - x, multiply by the bf16 pattern of 1.0); the i < j mask is
// applied only in the chunk that reaches the diagonal. A is loaded once per
// (wave, chunk), one chunk ahead, and reused by the 16 individuals of the
// workgroup, whose row labels are staged in LDS once per 1024 rows.
// FP32 accumulation is flushed into FP64 at every 256-row boundary, so no
// FP32 partial sum spans more than 256 rows.
#include "pga_internal.hpp"

#include <type_traits>

namespace pga {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t onehot2(uint32_t labs, uint32_t lj2) {
    const u16x2 x = __builtin_bit_cast(u16x2, labs ^ lj2);
    const u16x2 one = {1, 1};
    const u16x2 t = __builtin_elementwise_sub_sat(one, x);   // 1 where equal, else 0
    const u16x2 bf1 = {0x3F80, 0x3F80};                        // bf16 1.0
    return __builtin_bit_cast(uint32_t, t * bf1);
}

// One column block jb (64 stocks, 16 per wave) for the B individuals of batch pb.
__device__ __forceinline__ void mfma_block(const InstDesc &d, int jb, int pb, int parity,
                                           uint16_t (*lab_s)[kMfmaRowChunk]) {
    constexpr int B = kMfmaB;
    constexpr int RC = kMfmaRowChunk;
    const int N = d.N, P = d.P, ld = d.ld_h;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform, kept scalar
    const int lane = threadIdx.x & 63;
    const int n = lane & 15, g = lane >> 4;
    const int jt0 = jb * kMfmaCols + 16 * wave;
    const int j = jt0 + n;
    const int pbase = pb * B;
    const int32_t *__restrict__ labels = d.pop[parity];
    const uint16_t *__restrict__ hi = d.hi;
    const uint16_t *__restrict__ lo = d.lo;

    uint32_t lj2[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int p = pbase + b;
        const uint32_t l = (j < N && p < P) ? (uint32_t)gld(labels + (size_t)p * N + j) & 0xFFFFu : 0xFFFEu;
        lj2[b] = l | (l << 16);
    }
    floatx4 acc[B];
    double acc64[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        acc64[b] = 0.0;
    }
    const int dreg = n & 3;                                   // lane holds D[n][n] in register n & 3 ...
    const bool diag_lane = (n >> 2) == g;                     // ... when its 4-row group contains row n

    auto flush = [&]() {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const float v = dreg == 0 ? acc[b][0] : dreg == 1 ? acc[b][1] : dreg == 2 ? acc[b][2] : acc[b][3];
            acc64[b] += (double)v;
            acc[b] = floatx4{0.f, 0.f, 0.f, 0.f};
        }
    };
    auto load_a = [&](int i0, uint4 &ah, uint4 &al) {
        ah = make_uint4(0, 0, 0, 0);
        al = make_uint4(0, 0, 0, 0);
        if (j < ld) {
            ah = gld_u4(hi + (size_t)j * ld + i0 + 8 * g);
            al = gld_u4(lo + (size_t)j * ld + i0 + 8 * g);
        }
    };
    auto chunk = [&](auto masked_tag, int i0, int c0, uint4 ah, uint4 al) {
        constexpr bool masked = decltype(masked_tag)::value;
        const int ik = i0 + 8 * g;                            // first of this lane's 8 rows
        uint32_t m[4] = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
        if constexpr (masked) {
#pragma unroll
            for (int q = 0; q < 4; ++q)
                m[q] = ((ik + 2 * q < j) ? 0xFFFFu : 0u) | ((ik + 2 * q + 1 < j) ? 0xFFFF0000u : 0u);
        }
        const bf16x8 Ah = __builtin_bit_cast(bf16x8, ah);
        const bf16x8 Al = __builtin_bit_cast(bf16x8, al);
#pragma unroll
        for (int b = 0; b < B; b += 2) {
            const uint4 l0 = *(const uint4 *)&lab_s[b][ik - c0];
            const uint4 l1 = *(const uint4 *)&lab_s[b + 1][ik - c0];
            uint4 v0, v1;
            v0.x = onehot2(l0.x, lj2[b]);
            v0.y = onehot2(l0.y, lj2[b]);
            v0.z = onehot2(l0.z, lj2[b]);
            v0.w = onehot2(l0.w, lj2[b]);
            v1.x = onehot2(l1.x, lj2[b + 1]);
            v1.y = onehot2(l1.y, lj2[b + 1]);
            v1.z = onehot2(l1.z, lj2[b + 1]);
            v1.w = onehot2(l1.w, lj2[b + 1]);
            if constexpr (masked) {
                v0.x &= m[0]; v0.y &= m[1]; v0.z &= m[2]; v0.w &= m[3];
                v1.x &= m[0]; v1.y &= m[1]; v1.z &= m[2]; v1.w &= m[3];
            }
            const bf16x8 B0 = __builtin_bit_cast(bf16x8, v0);
            const bf16x8 B1 = __builtin_bit_cast(bf16x8, v1);
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B0, acc[b], 0, 0, 0);
            acc[b + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ah, B1, acc[b + 1], 0, 0, 0);
            acc[b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B0, acc[b], 0, 0, 0);
            acc[b + 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B1, acc[b + 1], 0, 0, 0);
        }
        if (((i0 + 32) % kMfmaFlushRows) == 0) flush();
    };

    const int wg_iend = min(jb * kMfmaCols + kMfmaCols, N);   // rows any wave of the group needs
    const int my_iend = jt0 < N ? min(jt0 + 16, N) : 0;       // rows this wave needs (i < j <= jt0+15)
    const int i_diag = (jt0 / 32) * 32;                       // first chunk that may hold i >= j

    for (int c0 = 0; c0 < wg_iend; c0 += RC) {
        const int rows = min(RC, wg_iend - c0);
        for (int e = threadIdx.x; e < B * RC; e += 256) {
            const int b = e / RC, r = e % RC;
            const int i = c0 + r, p = pbase + b;
            lab_s[b][r] = (r < rows && p < P) ? (uint16_t)gld(labels + (size_t)p * N + i) : (uint16_t)0xFFFFu;
        }
        __syncthreads();
        const int cend = min(c0 + RC, my_iend);
        if (c0 < cend) {
            uint4 ah, al, nh, nl;
            load_a(c0, ah, al);
            int i0 = c0;
            const int uend = min(cend, max(c0, i_diag));        // chunks entirely below the diagonal
            for (; i0 < uend; i0 += 32) {
                if (i0 + 32 < cend) load_a(i0 + 32, nh, nl);
                chunk(std::false_type{}, i0, c0, ah, al);
                ah = nh;
                al = nl;
            }
            for (; i0 < cend; i0 += 32) {
                if (i0 + 32 < cend) load_a(i0 + 32, nh, nl);
                chunk(std::true_type{}, i0, c0, ah, al);
                ah = nh;
                al = nl;
            }
        }
        __syncthreads();
    }
    flush();
    if (diag_lane && j < N) {
        const double cjj = gld(d.C + (size_t)j * N + j);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int p = pbase + b;
            if (p < P) gst(d.wsum + (size_t)p * N + j, fma(2.0, acc64[b], cjj));
        }
    }
}

// The triangle is folded: column blocks n_jb-1-jp and jp share a workgroup, so every
// workgroup processes the same number of row chunks.
__global__ __launch_bounds__(256) void k_pairsum_mfma(Tables t, int parity) {
    __shared__ __align__(16) uint16_t lab_s[kMfmaB][kMfmaRowChunk];
    const int tile = blockIdx.x;
    const int k = find_inst(t.tiles_mfma, t.n_inst, tile);
    const InstDesc &d = t.desc[k];
    const int local = tile - t.tiles_mfma[k];
    const int n_jb = (d.N + kMfmaCols - 1) / kMfmaCols;
    const int n_pairs = (n_jb + 1) / 2;
    const int jp = local % n_pairs;
    const int pb = local / n_pairs;
    mfma_block(d, n_jb - 1 - jp, pb, parity, lab_s);
    if (jp != n_jb - 1 - jp) {
        __syncthreads();
        mfma_block(d, jp, pb, parity, lab_s);
    }
}

hipError_t launch_pairsum_mfma(Tables t, int total_tiles, int parity, hipStream_t s) {
    if (total_tiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pairsum_mfma, dim3(total_tiles), dim3(256), 0, s, t, parity);
    return hipGetLastError();
}

}  // namespace pga
