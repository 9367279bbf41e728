// Size classes where the GA tuner's pick replaces the hand-coded defaults of
// EVOSORT_ALGO_AUTO for keys-only sorts (Sec. 4.2, Algorithm 2, run on an
// MI355X): key type (EVOSORT_* dtype code), size class (keys), the lengths
// lo <= n < hi the row applies to (geometric means with the neighbouring
// tuned size classes), A_code, tile threads, keys per thread (0, 0 for the
// mergesort).  Written by `python -m paper_2505_18681_amd.tuner
// --emit-header` from the packaged table tuned/mi355x.json; do not edit.
#pragma once

#include <stdint.h>

namespace evosort {

struct TunedRow {
    int dtype;
    int64_t n;
    int64_t lo;
    int64_t hi;
    int algo;
    int threads;
    int items;
};

constexpr TunedRow kTunedRows[] = {
    {1, 10000000, 3162278, 31622777, 4, 1024, 16},  // int32
    {2, 20000, 14143, 31623, 3, 0, 0},  // int64
    {2, 50000, 31623, 70711, 3, 0, 0},  // int64
    {2, 1000000, 447214, 3162278, 4, 1024, 8},  // int64
    {3, 1000000, 447214, 3162278, 4, 768, 12},  // uint32
    {3, 10000000, 3162278, 31622777, 4, 1024, 16},  // uint32
    {4, 10000000, 3162278, 31622777, 4, 1024, 20},  // float32
    {5, 20000, 14143, 31623, 3, 0, 0},  // float64
    {5, 50000, 31623, 70711, 3, 0, 0},  // float64
    {5, 100000, 70711, 141422, 3, 0, 0},  // float64
    {5, 1000000, 447214, 3162278, 4, 1024, 8},  // float64
};
constexpr int kTunedRowCount = 11;

}  // namespace evosort
