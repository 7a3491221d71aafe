// lcs_dist_build_noalloc: the single-pair build on a workspace that the
// library holds itself, for callers that cannot allocate device memory.
//
// The workspace is the file-scope device array `scratch` below: one copy per
// GPU, created with the code object and kept until the process ends.  In host
// code the array's name only stands for the symbol; its device address on the
// current GPU comes from hipGetSymbolAddress, looked up once per device and
// kept, and only that address is ever handed to a kernel.  Every call on a GPU
// shares that GPU's copy, so calls that overlap on one GPU race, and a build
// stays readable (length, trace, views) only until the next build on that GPU.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "lcs.h"

namespace {

constexpr size_t kScratchBytes = LCS_NOALLOC_WORKSPACE_BYTES;
__device__ __align__(256) uint8_t scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];  // device address of `scratch` per device; null until looked up

// Device address of the current GPU's copy of `scratch`.
int32_t scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return LCS_E_HIP;
    if (dev < 0 || dev >= kMaxDevices) return LCS_E_HIP;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LCS_E_HIP;
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return LCS_OK;
}

}  // namespace

extern "C" int32_t lcs_dist_build_noalloc(lcs_plan_t plan, const uint8_t *a, int32_t m,
                                          const uint8_t *b, int32_t n, void *stream) {
    if (!plan) return LCS_E_INVAL;
    size_t need = 0;
    int32_t rc = lcs_plan_workspace(plan, m, n, &need);
    if (rc != LCS_OK) return rc;
    if (need > kScratchBytes) return LCS_E_WORKSPACE;
    void *ws = nullptr;
    rc = scratch_address(&ws);
    if (rc != LCS_OK) return rc;
    return lcs_dist_build(plan, a, m, b, n, ws, kScratchBytes, stream);
}
