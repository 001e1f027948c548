// Allocation-free fitness entry point: pga_fitness whose scratch memory (the
// descriptor table, the per-stock pair sums, the scaled split copies, the
// route flags and the diagonal copy) lives in a static device array of this
// translation unit instead of a caller workspace.
//
// Host code never passes the array's name to a kernel or a copy: on the host
// that name is only a stand-in. Its device address is looked up once per
// device with hipGetSymbolAddress, with that device current, and kept; every
// launch then receives that address.
#include "pga_internal.hpp"

#include <mutex>

namespace {

constexpr size_t kScratchBytes = PGA_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call per device).
hipError_t scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

}  // namespace

extern "C" {

size_t pga_fitness_noalloc_max_bytes(void) { return kScratchBytes; }

int pga_fitness_noalloc(const double *C, const uint16_t *C_hi, const uint16_t *C_lo, int32_t N,
                        const int32_t *labels, int32_t P, int32_t form, double *fitness, int32_t *n_s,
                        double *c_s, int32_t *status, void *stream) {
    if (N < 1 || P < 0) return PGA_ERR_ARG;
    if (form != PGA_FORM_FP64 && form != PGA_FORM_BF16X2) return PGA_ERR_ARG;
    if (N > PGA_N_MAX) return PGA_ERR_UNSUPPORTED;
    if (P == 0) return PGA_OK;
    if (pga_fitness_ws_bytes(N, P, form) > kScratchBytes) return PGA_ERR_UNSUPPORTED;
    void *ws = nullptr;
    const hipError_t e = scratch_ptr(&ws);
    if (e != hipSuccess) {
        pga::note_hip_error((int)e);
        return PGA_ERR_HIP;
    }
    return pga::fitness_call(C, C_hi, C_lo, N, labels, P, form, fitness, n_s, c_s, status, ws, kScratchBytes,
                             (hipStream_t)stream, false);
}

}  // extern "C"
