// Bottom-up mergesort (Sec. 4, Algorithm 3) for gfx950: host-visible part.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <functional>

#include "kernels.hpp"

namespace evosort {

// Shape of one mergesort call.
struct MergePlan {
    int kb, vb;
    int64_t n;
    uint32_t t_ins;       // chunk length sorted before the first merge
    uint64_t block_keys;  // keys per block-sort workgroup: t_ins * 2^m <= capacity
    uint64_t block_run;   // == block_keys: sorted run length after the block sort
    uint64_t blocks;
    uint32_t rounds;      // global merge rounds until one run covers n
    uint32_t tile_out;    // outputs per merge workgroup
    uint64_t max_parts;   // partition entries needed by the largest round
};

MergePlan merge_plan(int kb, int vb, int64_t n, uint32_t t_ins);
size_t merge_partition_bytes(const MergePlan& mp);
// Partition entries one round with input runs of length `run` needs.
uint64_t merge_round_parts(const MergePlan& mp, int64_t run);
// Largest block the block sort holds for (kb, vb).
uint64_t merge_block_capacity(int kb, int vb);

struct MergeBlockArgs {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;
    void* vals_out;
    int64_t n;
    bool iota;       // values are input positions (argsort)
    bool skip_keys;  // do not write keys
};

struct MergeRoundArgs {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;
    void* vals_out;
    int64_t n;
    int64_t run;     // length of the sorted input runs
    int64_t* parts;  // merge-path split of every output tile
    bool skip_keys;
};

hipError_t launch_merge_block_sort(const KeyDesc& kd, int vb, const MergePlan& mp, const MergeBlockArgs& a,
                                   hipStream_t s);
hipError_t launch_merge_partition(const KeyDesc& kd, const MergePlan& mp, const MergeRoundArgs& a, hipStream_t s);
hipError_t launch_merge_round(const KeyDesc& kd, int vb, const MergePlan& mp, const MergeRoundArgs& a,
                              hipStream_t s);

struct MergeBuffers {
    const void* keys_in;
    void* keys_out;  // unused for argsort
    const void* vals_in;
    void* vals_out;  // values, or indices for argsort
    void* keys_tmp;
    void* keys_tmp2;  // argsort only
    void* vals_tmp;
    int64_t* parts;
    bool iota;  // argsort
};

// Launch hooks (so the caller can time each launch).
struct MergeLaunch {
    std::function<hipError_t(const MergeBlockArgs&)> block_sort;
    std::function<hipError_t(const MergeRoundArgs&)> partition;
    std::function<hipError_t(const MergeRoundArgs&)> merge;
};

// The whole mergesort: block sort, then `rounds` merge rounds, buffers
// alternating so that the last stage writes the outputs.
hipError_t run_merge_sort(const MergePlan& mp, const MergeBuffers& b, const MergeLaunch& ml);

}  // namespace evosort
