// Size classes where the GA tuner picked the mergesort over the radix sort
// for EVOSORT_ALGO_AUTO keys-only sorts (Sec. 4.2, Algorithm 2, run on an
// MI355X): key type (EVOSORT_* dtype code), size class (keys), the lengths
// lo <= n < hi the row applies to (geometric means with the neighbouring
// tuned size classes), A_code.  Written by `python -m
// paper_2505_18681_amd.tuner --emit-header` from the packaged table
// tuned/mi355x.json; do not edit.
#pragma once

#include <stdint.h>

namespace evosort {

struct TunedRow {
    int dtype;
    int64_t n;
    int64_t lo;
    int64_t hi;
    int algo;
};

constexpr TunedRow kTunedRows[] = {
    {2, 20000, 14143, 31623, 3},  // int64
    {2, 50000, 31623, 70711, 3},  // int64
    {5, 20000, 14143, 31623, 3},  // float64
    {5, 50000, 31623, 70711, 3},  // float64
};
constexpr int kTunedRowCount = 4;

}  // namespace evosort
