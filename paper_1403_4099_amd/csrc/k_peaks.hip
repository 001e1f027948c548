// Measurement aids: sustained bf16 MFMA throughput and FP64 vector FMA
// throughput of this GPU, the ceilings the pair-sum kernels' work is compared
// against beside the published peaks.
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

__global__ __launch_bounds__(256) void k_peak_mfma(float *out, int iters) {
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

}  // namespace pga
