// Tile shapes of the single-sweep radix pass, shared by the kernels and the
// host planner (no device code here).
#pragma once

#include <stddef.h>

#include "kernels.hpp"

namespace evosort {

// LDS per workgroup on gfx950.
constexpr size_t kLdsLimit = 160 * 1024;

// Static LDS of radix_pass_kernel<KB, VB, BITS, THREADS, ITEMS>: the union of
// the per-wave digit counters and lane buckets with the staging area, the
// per-digit output offsets, and a few words.
constexpr size_t radix_lds_bytes(int kb, int vb, int bits, int threads, int items)
{
    const size_t bins = (size_t)1 << bits;
    const size_t counters = (((size_t)(threads / 64) * bins * 4) + 15) & ~(size_t)15;
    const size_t hist = counters + (bits <= 11 ? (size_t)(threads / 64) * bins * 8 : 0);
    const size_t stage = (size_t)threads * items * (size_t)(kb + vb);
    return (hist > stage ? hist : stage) + bins * 8 + (size_t)(threads / 64) * 4 + 16;
}

// Waves per SIMD the pass kernel must keep so that registers do not cost it
// a workgroup that LDS would allow on a CU (4 SIMDs per CU), at most 6 (80
// VGPRs, which the pass fits in): the compiler is held to this bound.
constexpr int radix_pass_waves_per_eu(int kb, int vb, int bits, int threads, int items)
{
    const size_t lds = radix_lds_bytes(kb, vb, bits, threads, items);
    const int groups = lds > 0 ? (int)(kLdsLimit / lds) : 1;
    const int waves = (groups < 1 ? 1 : groups) * (threads / 64);
    const int per_eu = (waves + 3) / 4;
    return per_eu > 6 ? 6 : (per_eu < 1 ? 1 : per_eu);
}

// Preferred shape per (key bytes, value bytes), measured at 8-bit digits on
// 1e9-key arrays; compiled at every digit width (used where it fits in LDS).
// The GA tuner's pick of 16-wave, 16384-key tiles over the earlier 8-wave,
// 12288-key ones led to a sweep of 12- and 16-wave shapes: 12-wave tiles of
// 24 keys per thread for 4-byte keys (18432 keys, 74 KB of LDS, two
// workgroups per CU) and of 12 for 8-byte keys are 8 % and 3 % faster than
// the 8-wave defaults they replace.  Fewer, larger tiles cut the look-back
// traffic and lengthen the runs of each digit in the write-out.
constexpr RadixShape radix_default_shape_c(int kb, int vb)
{
    // keys-only and 4-byte values of 4-byte keys; 8-byte values; 8-byte keys
    if (kb == 4)
        return vb == 8 ? RadixShape{512, 24} : RadixShape{768, 24};
    if (vb == 0)
        return RadixShape{768, 12};
    return vb == 4 ? RadixShape{512, 24} : RadixShape{512, 16};
}

// Shape used when the preferred one does not fit at a digit width; compiled
// at every digit width and fits in LDS at all of them.
constexpr RadixShape kRadixFallbackShape{256, 8};

// Alternative shapes, compiled at digit width 8 only (those that fit in LDS).
#define EVOSORT_RADIX_ALT_SHAPES(X)                                                                          \
    X(256, 8) X(256, 12) X(256, 16) X(256, 24) X(256, 32) X(256, 48) X(512, 8) X(512, 16) X(512, 24) X(512, 32) \
    X(768, 12) X(768, 16) X(768, 20) X(768, 24) X(1024, 8) X(1024, 12) X(1024, 16) X(1024, 20)

// Tile shapes of the segmented pass (8-bit digits, 32-bit look-back words),
// compiled where they fit in LDS.
#define EVOSORT_SEG_SHAPES(X) X(512, 24) X(1024, 16) X(512, 16) X(256, 16) X(256, 8) X(768, 24) X(768, 12)

}  // namespace evosort
