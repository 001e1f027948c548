// Measurement aids: sustained bf16 MFMA throughput and FP64 vector FMA
// throughput of this GPU, the ceilings the pair-sum kernels' work is compared
// against beside the published peaks; and the pipe-mix loops, which time MFMA,
// vector ALU and LDS work alone and together on one SIMD.
//
// MFMA: Each wave issues `iters` rounds of 16 independent
// v_mfma_f32_16x16x32_bf16 (16 384 flops each) on register operands and
// writes one sum per wave, so nothing but the MFMA pipe is exercised. Sixteen
// accumulation chains per wave are needed to reach the pipe's rate: with eight,
// each MFMA waits on its chain's previous result and the rate stays near 60%.
#include "pga_internal.hpp"

namespace pga {

typedef __bf16 bf16x8_p __attribute__((ext_vector_type(8)));
typedef float floatx4_p __attribute__((ext_vector_type(4)));

constexpr int kPeakChains = 16;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_peak_mfma(float *out, int iters) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    // operands near 2^-7 (bf16 0x3C00 plus a lane-dependent mantissa): sums stay small and finite
    const uint32_t w = 0x3C003C00u + (uint32_t)(lane & 7) * 0x00010001u;
    const bf16x8_p a = __builtin_bit_cast(bf16x8_p, uint4{w, w ^ 0x00010000u, w, w});
    const bf16x8_p b = __builtin_bit_cast(bf16x8_p, uint4{w, w, w ^ 0x00000001u, w});
    floatx4_p acc[kPeakChains];
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) acc[k] = floatx4_p{0.f, 0.f, 0.f, 0.f};
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kPeakChains; ++k) acc[k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[k], 0, 0, 0);
    }
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < kPeakChains; ++k) s += acc[k][0] + acc[k][1] + acc[k][2] + acc[k][3];
    if (lane == 0) out[(size_t)blockIdx.x * 4 + wave] = s;
}

// FP64 vector ceiling: every lane runs kFmaChains independent FP64 FMA chains
// (v_fma_f64, 2 flops per lane per instruction) on register operands; the
// multiplier is just below 1 so the values stay finite and the compiler cannot
// fold the loop.
constexpr int kFmaChains = 8;

__global__ __launch_bounds__(256) void k_peak_fp64(double *out, int iters, double m) {
    double acc[kFmaChains];
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) acc[k] = (double)(threadIdx.x + k);
    const double c = 1.0 / 1024.0;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int k = 0; k < kFmaChains; ++k) acc[k] = fma(acc[k], m, c);
    }
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kFmaChains; ++k) s += acc[k];
    if ((threadIdx.x & 63) == 0) out[(size_t)blockIdx.x * 4 + (threadIdx.x >> 6)] = s;
}

hipError_t launch_peak_fp64(double *out, int n_workgroups, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_fp64, dim3(n_workgroups), dim3(256), 0, s, out, iters, 0.999);
    return hipGetLastError();
}

double peak_fp64_flops(int n_workgroups, int iters) {
    return (double)n_workgroups * 256.0 * (double)iters * kFmaChains * 2.0;
}

hipError_t launch_peak_mfma(float *out, int n_workgroups, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_mfma, dim3(n_workgroups), dim3(256), 0, s, out, iters);
    return hipGetLastError();
}

double peak_mfma_flops(int n_workgroups, int iters) {
    return (double)n_workgroups * 4.0 * (double)iters * kPeakChains * 16384.0;
}


// Pipe mix. Every wave runs `iters` rounds of the work `mode` selects:
//   kMixMfma  4 independent v_mfma_f32_16x16x32_bf16 (one individual's hi and lo
//             products for two chunks, as in the pair-sum kernels);
//   kMixValu  the one-hot of one individual's B operand as the register
//             column kernel builds it: 4 DPP-broadcast xors and 4 saturating
//             16-bit subtracts, in 4 dependent chains;
//   kMixLds   2 ds_read_b128 of conflict-free addresses (a 4 KB table); with
//             kMixMfma the data are the MFMAs' B operands, alone each read is
//             folded into a sink with one xor;
//   kMixSplit even waves do the MFMA work, odd waves the rest.
// Comparing the time of the work together with the times of its parts shows
// which pipes of a SIMD overlap. One float per wave goes to out.
constexpr int kMixMfma = 1, kMixValu = 2, kMixLds = 4, kMixSplit = 8;

template <int B>
__device__ __forceinline__ uint32_t mix_bcast(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x150 + B, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t mix_onehot(uint32_t r, uint32_t c) {
    typedef unsigned short u16x2_p __attribute__((ext_vector_type(2)));
    const u16x2_p x = __builtin_bit_cast(u16x2_p, r ^ c);
    const u16x2_p one = {0x0100, 0x0100};
    return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(one, x));
}

template <int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8))) void k_pipe_mix(float *out, int iters) {
    __shared__ __align__(16) pga_u32x4 tab[256];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar branches
    tab[threadIdx.x] = pga_u32x4{threadIdx.x, threadIdx.x ^ 1u, 0x3C003C00u, 0x3C003C00u};
    __syncthreads();
    constexpr bool split = (MODE & kMixSplit) != 0;
    const bool do_m = (MODE & kMixMfma) && (!split || (wave & 1) == 0);
    const bool do_v = (MODE & kMixValu) && (!split || (wave & 1) == 1);
    const bool do_l = (MODE & kMixLds) && (!split || (wave & 1) == 1 || !(MODE & kMixValu));
    const uint32_t w = 0x3C003C00u + (uint32_t)(lane & 7) * 0x00010001u;
    const bf16x8_p a = __builtin_bit_cast(bf16x8_p, uint4{w, w ^ 0x00010000u, w, w});
    bf16x8_p b0 = __builtin_bit_cast(bf16x8_p, uint4{w, w, w ^ 0x00000001u, w});
    bf16x8_p b1 = b0;
    floatx4_p acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = acc0, acc2 = acc0, acc3 = acc0;
    uint32_t r0 = (uint32_t)lane << 8, r1 = r0 ^ 0x100u, r2 = r0 ^ 0x200u, r3 = r0 ^ 0x300u;
    const uint32_t col = (uint32_t)(lane & 15) << 8 | (uint32_t)(lane & 15) << 24;
    uint32_t sink = 0;
    const volatile __attribute__((address_space(3))) pga_u32x4 *tp =
        (const volatile __attribute__((address_space(3))) pga_u32x4 *)tab;
    for (int it = 0; it < iters; ++it) {
        if (do_l) {
            const pga_u32x4 x0 = tp[lane], x1 = tp[64 + lane];
            if (do_m) {
                b0 = __builtin_bit_cast(bf16x8_p, x0);
                b1 = __builtin_bit_cast(bf16x8_p, x1);
            } else {
                sink ^= x0.x ^ x1.y;
            }
        }
        if (do_m) {
            acc0 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc3, 0, 0, 0);
        }
        if (do_v) {
            r0 = mix_onehot(mix_bcast<0>(r0), col);
            r1 = mix_onehot(mix_bcast<1>(r1), col);
            r2 = mix_onehot(mix_bcast<2>(r2), col);
            r3 = mix_onehot(mix_bcast<3>(r3), col);
        }
    }
    const float s = (float)(sink ^ r0 ^ r1 ^ r2 ^ r3) + acc0[0] + acc1[1] + acc2[2] + acc3[3];
    if (lane == 0) out[(size_t)blockIdx.x * 4 + wave] = s;
}

hipError_t launch_pipe_mix(float *out, int mode, int n_workgroups, int iters, hipStream_t s) {
    switch (mode) {
#define PGA_MIX(m)                                                                                       \
    case m:                                                                                              \
        hipLaunchKernelGGL(k_pipe_mix<m>, dim3(n_workgroups), dim3(256), 0, s, out, iters);              \
        break;
        PGA_MIX(1) PGA_MIX(2) PGA_MIX(3) PGA_MIX(4) PGA_MIX(5) PGA_MIX(11) PGA_MIX(13)
#undef PGA_MIX
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pga
