// One-workgroup sort of small arrays (host-visible part).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace evosort {

// Largest n the one-workgroup sort takes: the whole array (keys and values,
// or indices) stays in one workgroup's registers and LDS for every pass.
constexpr int kSmallCapacity = 16384;    // 4-byte keys; 8-byte keys without values
constexpr int kSmallCapacity8V = 8192;   // 8-byte keys with values or indices

enum SmallMode : int { SMALL_MODE_KEYS = 0, SMALL_MODE_PAIRS = 1, SMALL_MODE_ARGSORT = 2 };

struct SmallSortArgs {
    const void* keys_in;
    void* keys_out;       // unused for argsort
    const void* vals_in;  // pairs only
    void* vals_out;       // values (pairs) or indices (argsort)
    int64_t n;
    int mode;
    uint32_t* error_word;  // cleared by the kernel (no device-side error can occur here); may be null
};

int64_t small_sort_capacity(int key_bytes, int val_bytes);
hipError_t launch_small_sort(const KeyDesc& kd, int val_bytes, const SmallSortArgs& a, hipStream_t s);

}  // namespace evosort
