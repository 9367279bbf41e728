// Size classes where the GA tuner's pick replaces the hand-coded defaults of
// EVOSORT_ALGO_AUTO for keys-only sorts (Sec. 4.2, Algorithm 2, run on an
// MI355X): key bytes, size class (keys), A_code, tile threads, keys per thread.
// A row applies to arrays within half a decade of its size class.  Written by
// `python -m paper_2505_18681_amd.tuner --emit-header` from the packaged
// table tuned/mi355x.json; do not edit.
#pragma once

#include <stdint.h>

namespace evosort {

struct TunedRow {
    int key_bytes;
    int64_t n;
    int algo;
    int threads;
    int items;
};

constexpr TunedRow kTunedRows[] = {
    {4, 10000000, 4, 1024, 16},
};
constexpr int kTunedRowCount = 1;

}  // namespace evosort
