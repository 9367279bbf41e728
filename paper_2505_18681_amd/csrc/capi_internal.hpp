// Entry points of the library used by its own server (not exported): the
// public sorts without the report of an earlier call's pending device error,
// with the host-visible error word chosen by the caller (the server gives
// each stream slot its own word, so a failure is charged to the job that had
// it).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "evosort.h"

namespace evosort {

evosort_status server_sort(int dtype, const void* keys_in, void* keys_out, int64_t n, void* temp,
                           size_t temp_bytes, const evosort_params* p, hipStream_t s, uint32_t* host_error);

evosort_status server_segmented_sort(int dtype, const void* keys_in, void* keys_out, int64_t n,
                                     const int64_t* offsets, int64_t nseg, void* temp, size_t temp_bytes,
                                     const evosort_params* p, hipStream_t s, uint32_t* host_error);

// Status of a device error word's bits (0: EVOSORT_OK).
evosort_status status_of_error_bits(uint32_t bits);

// evosort_sort with its scratch at `scratch` (scratch_bytes long): reports an
// earlier call's pending device error first, returns
// EVOSORT_ERR_TEMP_TOO_SMALL when the sort needs more scratch, and creates,
// allocates and frees nothing (no profiling events either).
evosort_status sort_in_scratch(int dtype, const void* keys_in, void* keys_out, int64_t n, const evosort_params* p,
                               hipStream_t s, void* scratch, size_t scratch_bytes);

// Records e as this thread's last HIP error; returns EVOSORT_ERR_HIP.
evosort_status record_hip_failure(hipError_t e);

}  // namespace evosort
