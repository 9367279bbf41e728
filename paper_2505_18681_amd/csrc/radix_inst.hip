// Instantiations of the single-sweep radix pass for one (key bytes, value
// bytes) pair.  The build compiles this file once per pair with
// -DEVOSORT_KB=<4|8> -DEVOSORT_VB=<0|4|8>, so the six pairs compile in
// parallel.
//
// Compiled set: the preferred and the fallback tile shape at every digit
// width 4..12, plus the alternative tile shapes at digit width 8; each with
// 32-bit look-back words (n < 2^30) and 64-bit ones.
#include "radix_impl.hpp"
#include "radix_shapes.hpp"

#ifndef EVOSORT_KB
#error "EVOSORT_KB must be defined"
#endif
#ifndef EVOSORT_VB
#error "EVOSORT_VB must be defined"
#endif

#define EVOSORT_CAT4(a, b, c, d) a##b##c##d
#define EVOSORT_XCAT4(a, b, c, d) EVOSORT_CAT4(a, b, c, d)
#define EVOSORT_NAME(kb, vb) EVOSORT_XCAT4(radix_pass_dispatch_k, kb, _v, vb)
#define EVOSORT_SEG_NAME(kb, vb) EVOSORT_XCAT4(seg_pass_dispatch_k, kb, _v, vb)

namespace evosort {

namespace {

template <int THREADS, int ITEMS, typename ST, int BITS>
hipError_t one(int bits, const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles, hipStream_t s, bool* found)
{
    if constexpr (BITS > 12) {
        (void)bits;
        (void)kd;
        (void)a;
        (void)tiles;
        (void)s;
        (void)found;
        return hipSuccess;
    } else {
        if (bits == BITS) {
            if constexpr (radix_lds_bytes(EVOSORT_KB, EVOSORT_VB, BITS, THREADS, ITEMS) <= kLdsLimit) {
                *found = true;
                return launch_radix_pass_t<EVOSORT_KB, EVOSORT_VB, BITS, THREADS, ITEMS, ST>(kd, a, tiles, s);
            } else {
                return hipSuccess;
            }
        }
        return one<THREADS, ITEMS, ST, BITS + 1>(bits, kd, a, tiles, s, found);
    }
}

template <int THREADS, int ITEMS, typename ST>
hipError_t all_bits(int bits, const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles, hipStream_t s,
                    bool* found)
{
    return one<THREADS, ITEMS, ST, 4>(bits, kd, a, tiles, s, found);
}

template <int THREADS, int ITEMS, typename ST>
hipError_t bits8(int bits, const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles, hipStream_t s, bool* found)
{
    if (bits != 8)
        return hipSuccess;
    if constexpr (radix_lds_bytes(EVOSORT_KB, EVOSORT_VB, 8, THREADS, ITEMS) <= kLdsLimit) {
        *found = true;
        return launch_radix_pass_t<EVOSORT_KB, EVOSORT_VB, 8, THREADS, ITEMS, ST>(kd, a, tiles, s);
    }
    return hipSuccess;
}

template <typename ST>
hipError_t by_shape(int bits, RadixShape sh, const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles,
                    hipStream_t s, bool* found)
{
    constexpr RadixShape def = radix_default_shape_c(EVOSORT_KB, EVOSORT_VB);
    if (sh.threads == def.threads && sh.items == def.items)
        return all_bits<def.threads, def.items, ST>(bits, kd, a, tiles, s, found);
    if (sh.threads == kRadixFallbackShape.threads && sh.items == kRadixFallbackShape.items)
        return all_bits<kRadixFallbackShape.threads, kRadixFallbackShape.items, ST>(bits, kd, a, tiles, s, found);
#define EVOSORT_TRY_SHAPE(T, I)                                  \
    if (sh.threads == (T) && sh.items == (I))                    \
        return bits8<(T), (I), ST>(bits, kd, a, tiles, s, found);
    EVOSORT_RADIX_ALT_SHAPES(EVOSORT_TRY_SHAPE)
#undef EVOSORT_TRY_SHAPE
    return hipSuccess;
}

}  // namespace

// Launches the pass kernel for (EVOSORT_KB, EVOSORT_VB); *found tells whether
// the requested (bits, shape, status width) is compiled in.
hipError_t EVOSORT_NAME(EVOSORT_KB, EVOSORT_VB)(int bits, RadixShape sh, int status_bytes, const KeyDesc& kd,
                                                 const RadixPassArgs& a, uint32_t tiles, hipStream_t s,
                                                 bool* found)
{
    *found = false;
    if (status_bytes == 4)
        return by_shape<uint32_t>(bits, sh, kd, a, tiles, s, found);
    if (status_bytes == 8)
        return by_shape<uint64_t>(bits, sh, kd, a, tiles, s, found);
    return hipSuccess;
}

// Segmented pass for (EVOSORT_KB, EVOSORT_VB) at 8-bit digits; *found tells
// whether the shape is compiled in.
hipError_t EVOSORT_SEG_NAME(EVOSORT_KB, EVOSORT_VB)(RadixShape sh, const KeyDesc& kd, const SegPassArgs& a,
                                                     uint32_t grid, hipStream_t s, bool* found)
{
    *found = false;
#define EVOSORT_TRY_SEG_SHAPE(T, I)                                                                     \
    if constexpr (radix_lds_bytes(EVOSORT_KB, EVOSORT_VB, kSegBits, (T), (I)) <= kLdsLimit) {           \
        if (sh.threads == (T) && sh.items == (I)) {                                                     \
            *found = true;                                                                              \
            return launch_seg_radix_pass_t<EVOSORT_KB, EVOSORT_VB, kSegBits, (T), (I)>(kd, a, grid, s); \
        }                                                                                               \
    }
    EVOSORT_SEG_SHAPES(EVOSORT_TRY_SEG_SHAPE)
#undef EVOSORT_TRY_SEG_SHAPE
    return hipSuccess;
}

}  // namespace evosort
