// Tile shapes of the single-sweep radix pass, shared by the kernels and the
// host planner (no device code here).
#pragma once

#include <stddef.h>

#include "kernels.hpp"

namespace evosort {

// LDS per workgroup on gfx950.
constexpr size_t kLdsLimit = 160 * 1024;

// Static LDS of radix_pass_kernel<KB, VB, BITS, THREADS, ITEMS>: the union of
// the per-wave digit counters and the staging area, the per-digit output
// offsets, and a few words.
constexpr size_t radix_lds_bytes(int kb, int vb, int bits, int threads, int items)
{
    const size_t bins = (size_t)1 << bits;
    const size_t hist = (size_t)(threads / 64) * bins * 4;
    const size_t stage = (size_t)threads * items * (size_t)(kb + vb);
    return (hist > stage ? hist : stage) + bins * 8 + (size_t)(threads / 64) * 4 + 16;
}

// Default shape per (key bytes, value bytes): compiled at every digit width.
constexpr RadixShape radix_default_shape_c(int kb, int vb)
{
    return (kb + vb) >= 16 ? RadixShape{256, 12} : RadixShape{256, 16};
}

// Alternative shapes, compiled at digit width 8 only (those that fit in LDS).
#define EVOSORT_RADIX_ALT_SHAPES(X) X(256, 8) X(256, 12) X(256, 16) X(256, 24) X(256, 32) X(512, 8) X(512, 16)

}  // namespace evosort
