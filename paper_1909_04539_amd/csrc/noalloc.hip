// The mixed-precision solve for callers that cannot allocate device memory
// (code under HIP graph capture, serving loops, harnesses that forbid
// hipMalloc): the FP32 residual scratch of the multi-pass form lives in a
// file-scope device array instead of a caller workspace.
//
// In host code `scratch` names a host-side stand-in, not device memory; its
// device address is taken once per device with hipGetSymbolAddress (with that
// device current) and only that address is passed to kernels.
#include <mutex>

#include "internal.h"

namespace sbs {
namespace {

constexpr size_t kStaticScratchBytes = size_t(64) << 20;  // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// Device address of this device's copy of `scratch` (nullptr on failure).
void *scratch_ptr(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        g_ptr[dev] = p;
    }
    return g_ptr[dev];
}

}  // namespace
}  // namespace sbs

using namespace sbs;

extern "C" {

size_t sbs_refined_static_scratch_bytes(void) { return kStaticScratchBytes; }

sbs_status sbs_solve_batch_refined_noalloc(sbs_handle h, const float *b, double *x, int64_t m, int32_t sweeps,
                                           void *stream) {
    const sbs_status st = refined_check(h, b, x, m, sweeps);
    if (st != SBS_OK || m == 0) return st;
    float *r = nullptr;
    if (!refined_fused(h, m)) {
        if (sbs_refined_workspace_bytes(h, m) > kStaticScratchBytes) return SBS_ERR_INVALID_ARG;
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess) return SBS_ERR_DEVICE;
        r = static_cast<float *>(scratch_ptr(dev));
        if (!r) return SBS_ERR_DEVICE;
    }
    return refined_run(h, b, x, m, sweeps, r, static_cast<hipStream_t>(stream));
}

}  // extern "C"
