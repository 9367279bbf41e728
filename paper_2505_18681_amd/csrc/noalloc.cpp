// The allocation-free sort entry point: evosort_sort with its scratch in a
// file-scope device array instead of a caller's buffer, for callers that
// cannot allocate (code under HIP graph capture, tight serving loops).
//
// `scratch` below is a host-side stand-in for a device symbol: every device
// that loads the library holds its own copy of the array, at its own address,
// until the process ends.  Host code never hands the stand-in to a kernel or a
// copy; it asks the runtime for the current device's address once per device
// (hipGetSymbolAddress, with that device current) and uses that address from
// then on.
#include <hip/hip_runtime.h>

#include <mutex>

#include "capi_internal.hpp"
#include "evosort.h"

namespace {

constexpr size_t kScratchBytes = EVOSORT_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "whole 256-byte blocks");

// The scratch of every allocation-free sort on a device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_dev[kMaxDevices];  // device address of `scratch` per device; null until looked up

// The current device's address of `scratch` (looked up on the first call on
// that device).  No allocation: a fixed table, one lookup per device.
evosort_status scratch_address(void** out)
{
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess)
        return evosort::record_hip_failure(e);
    if (dev < 0 || dev >= kMaxDevices)
        return EVOSORT_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_scratch_dev[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return evosort::record_hip_failure(e != hipSuccess ? e : hipErrorInvalidSymbol);
        g_scratch_dev[dev] = p;
    }
    *out = g_scratch_dev[dev];
    return EVOSORT_OK;
}

}  // namespace

extern "C" evosort_status evosort_sort_noalloc(int dtype, const void* keys_in, void* keys_out, int64_t n,
                                               const evosort_params* p, void* stream)
{
    void* ptr = nullptr;
    const evosort_status st = scratch_address(&ptr);
    if (st != EVOSORT_OK)
        return st;
    return evosort::sort_in_scratch(dtype, keys_in, keys_out, n, p, reinterpret_cast<hipStream_t>(stream), ptr,
                                    kScratchBytes);
}
