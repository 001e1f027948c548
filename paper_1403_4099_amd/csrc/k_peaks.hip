// Measurement aid: sustained bf16 MFMA throughput of this GPU, the ceiling the
// pair-sum kernel's issued MFMA work is compared against beside the published
// peak. Each wave issues `iters` rounds of 16 independent
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

hipError_t launch_peak_mfma(float *out, int n_workgroups, int iters, hipStream_t s) {
    hipLaunchKernelGGL(k_peak_mfma, dim3(n_workgroups), dim3(256), 0, s, out, iters);
    return hipGetLastError();
}

double peak_mfma_flops(int n_workgroups, int iters) {
    return (double)n_workgroups * 4.0 * (double)iters * kPeakChains * 16384.0;
}

}  // namespace pga
