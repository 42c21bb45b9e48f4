// dpm_moments_noalloc: dpm_moments_async for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid it).  Its
// power table and workspace live in one fixed device array of this file, `scratch`,
// which each GPU holds for the life of the process; the call allocates and frees
// nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "../../include/dpm.h"
#include "dpm_common.h"

namespace dpm {
int moments_in_scratch(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                       const dpm_out *out_device, uint8_t *scratch, size_t scratch_bytes, hipStream_t st,
                       size_t *need);  // dpm_api.cpp
}  // namespace dpm

namespace {

// One copy per GPU.  In host code the name is only a stand-in for the symbol: its device
// address, per device, comes from hipGetSymbolAddress below and is all that is passed on.
__device__ __align__(256) uint8_t scratch[DPM_NOALLOC_SCRATCH_BYTES];

std::mutex g_mu;
void *g_scratch_dev[64] = {};  // device address of `scratch` on each device

// Device address of this device's copy of `scratch`, looked up once per device with
// that device current.
int scratch_address(uint8_t **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return DPM_EDEVICE;
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) return DPM_EDEVICE;
        g_scratch_dev[dev] = ptr;
    }
    *out = static_cast<uint8_t *>(g_scratch_dev[dev]);
    return DPM_OK;
}

}  // namespace

extern "C" {

int dpm_moments_noalloc(const void *volume, const int64_t dims[3], dpm_dtype dtype, int max_order,
                        const dpm_out *out_device, void *stream, size_t *scratch_needed) {
    if (scratch_needed) *scratch_needed = 0;
    if (!volume || !out_device) return DPM_EINVAL;
    uint8_t *base = nullptr;
    int rc = scratch_address(&base);
    if (rc) return rc;
    return dpm::moments_in_scratch(volume, dims, dtype, max_order, out_device, base, DPM_NOALLOC_SCRATCH_BYTES,
                                   static_cast<hipStream_t>(stream), scratch_needed);
}

size_t dpm_noalloc_scratch_bytes(void) { return DPM_NOALLOC_SCRATCH_BYTES; }

}  // extern "C"
