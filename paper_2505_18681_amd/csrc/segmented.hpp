// Batched segmented sort: many independent arrays (segments) of one buffer
// sorted by one fixed sequence of launches, with every decision that depends
// on the segment sizes taken on the device.  No host synchronisation, no
// allocation and no memset, so the sequence can be captured in a HIP graph and
// replayed with new offsets.
//
//   seg_validate      offsets non-decreasing within [0, n] (else nothing is
//                     sorted and the error word says so);
//   seg_classify      each segment goes to a size class: a one-workgroup
//                     class (the whole segment sorted in LDS) or the large
//                     class (tiles of the single-sweep radix pass); class
//                     lists and the tiles of large segments are appended
//                     with wave-aggregated atomics;
//   seg_setup         per large segment: zero its digit histogram, write the
//                     tile -> segment map;
//   seg_histogram     digit histograms of every pass of every large segment
//                     (one read), zeroes the look-back words of its tiles;
//   seg_scan          per large segment and pass: digit bases;
//   seg_block_sort    persistent workgroups take small segments from their
//                     class list and sort each in LDS by 8-bit LSD passes;
//   seg_radix_pass    one single-sweep pass over all tiles of all large
//                     segments; a segment's first tile starts its own
//                     look-back chain.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "kernels.hpp"

namespace evosort {

// Digit width of the segmented routine (the paper's 8-bit digits).
constexpr int kSegBits = 8;
constexpr int kSegBins = 1 << kSegBits;

// One-workgroup classes for records of rb = key bytes + value bytes:
// workgroup size and keys per thread; capacities ascend.
struct SegClass {
    int threads;
    int items;
};
constexpr int kSegMaxClasses = 4;
constexpr int seg_class_count(int rb) { return rb == 4 ? 4 : 3; }
constexpr SegClass seg_class(int rb, int c)
{
    return c == 0   ? SegClass{64, 8}
           : c == 1 ? SegClass{256, 8}
           : c == 2 ? (rb <= 8 ? SegClass{512, 16} : SegClass{512, 8})
                    : SegClass{1024, 16};
}
constexpr int64_t seg_class_capacity(int rb, int c) { return (int64_t)seg_class(rb, c).threads * seg_class(rb, c).items; }
constexpr int64_t seg_block_capacity(int rb) { return seg_class_capacity(rb, seg_class_count(rb) - 1); }

// Bits of the device error word.
constexpr uint32_t kDeviceErrTimeout = 1u;     // a look-back wait ran out of its spin limit
constexpr uint32_t kDeviceErrBadSegment = 2u;  // offsets not non-decreasing within [0, n], or a segment >= 2^30 keys

// A large segment: its keys and its range of tiles.
struct SegLarge {
    int64_t begin;
    uint32_t len;
    uint32_t first_tile;
};

// Device words in the scratch header, all zeroed at the start of each call.
struct SegCounters {
    uint32_t class_count[kSegMaxClasses + 1];  // [kSegMaxClasses]: large segments
    uint32_t tile_count;
    uint32_t class_ticket[kSegMaxClasses];
    uint32_t pass_ticket[8];
};

struct SegClassifyArgs {
    const int64_t* offsets;  // nseg + 1
    int64_t nseg;
    int64_t n;
    int64_t block_limit;  // segments shorter than this (and not empty) take a one-workgroup class
    int classes;
    int64_t cap[kSegMaxClasses];
    uint32_t tile_keys;
    SegCounters* ctr;
    uint32_t* lists;  // (classes + 1) lists of nseg entries
    SegLarge* large;
    uint32_t* error_word;
    uint32_t* host_error;  // host-visible word also set when the offsets are bad (may be null)
};

// Per-large-segment kernels walk slots [0, *nlarge) with a grid stride.
struct SegLargeArgs {
    const uint32_t* nlarge;
    const SegLarge* large;
    uint32_t* tile_slot;
    uint32_t* hist;   // per slot: passes * 256 counts
    uint64_t* bases;  // per slot: passes * 256 first output slots (relative to the segment)
    int passes;
};

struct SegHistArgs {
    const void* keys;
    const uint32_t* tile_count;
    const SegLarge* large;
    const uint32_t* tile_slot;
    uint32_t* hist;
    uint32_t* status;         // passes arrays of status_pass_words look-back words
    size_t status_pass_words;
    uint32_t tile_keys;
    uint32_t group;           // tiles per workgroup
    int passes;
};

struct SegBlockArgs {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;
    void* vals_out;
    const int64_t* offsets;
    const uint32_t* list;
    const uint32_t* count;
    uint32_t* ticket;
};

// Arguments of one segmented radix pass: `base` holds the whole-buffer
// pointers, the pass's shift, flags and spin limit; `base.bases` points at
// slot 0's bases of this pass (slot stride slot_stride words) and
// `base.status` at this pass's look-back words (indexed by global tile).
struct SegPassArgs {
    RadixPassArgs base;
    const uint32_t* tile_slot;
    const SegLarge* large;
    const uint32_t* tile_count;
    uint32_t slot_stride;
};

hipError_t launch_seg_classify(const SegClassifyArgs& a, hipStream_t s);
hipError_t launch_seg_setup(const SegLargeArgs& a, uint32_t tile_keys, uint32_t grid, hipStream_t s);
hipError_t launch_seg_histogram(const KeyDesc& kd, const SegHistArgs& a, uint32_t grid, hipStream_t s);
hipError_t launch_seg_scan(const SegLargeArgs& a, uint32_t grid, hipStream_t s);
// One launch per class: persistent workgroups, at most max_grid of them and
// no more than fit on the device at once.
hipError_t launch_seg_block_sort(const KeyDesc& kd, int val_bytes, int cls, const SegBlockArgs& a,
                                 uint32_t max_grid, hipStream_t s);

// Segmented radix pass (8-bit digits, 32-bit look-back words).
bool seg_pass_available(int key_bytes, int val_bytes, RadixShape shape);
RadixShape seg_default_shape(int key_bytes, int val_bytes);
hipError_t launch_seg_radix_pass(const KeyDesc& kd, int val_bytes, RadixShape shape, const SegPassArgs& a,
                                 uint32_t grid, hipStream_t s);

}  // namespace evosort
