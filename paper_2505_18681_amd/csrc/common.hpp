// Device helpers shared by the radix and merge kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace evosort {

constexpr int kWave = 64;

template <int KB>
struct KeyWord;
template <>
struct KeyWord<4> {
    using U = uint32_t;
};
template <>
struct KeyWord<8> {
    using U = uint64_t;
};

template <int VB>
struct ValWord {
    using T = uint32_t;  // placeholder when there are no values
};
template <>
struct ValWord<8> {
    using T = uint64_t;
};

// Order map of a key type: an unsigned word whose natural order is the key
// order.  For a key word k with sign bit s (all-ones word when set):
//   to_order(k) = k ^ (flip | (s & neg))
// signed ints: flip = sign bit, neg = 0 (the paper's sign-bit XOR, Sec. 4,
// Algorithms 4 and 5); uint32: flip = neg = 0; IEEE floats: flip = sign bit,
// neg = all ones, so negative values are complemented (totalOrder).
// The keys themselves are never rewritten: the map is applied on every load
// that needs a digit or a comparison, and original bits are what gets stored.
// Descending order complements the order word (desc = all ones): the stable
// sort of the complemented words is the descending stable sort.
template <typename U>
struct OrderMap {
    U flip;
    U neg;
    U desc;

    __device__ __forceinline__ U sign_word(U k) const
    {
        using S = std::make_signed_t<U>;
        return (U)((S)k >> (sizeof(U) * 8 - 1));
    }
    __device__ __forceinline__ U to_order(U k) const { return (k ^ (flip | (sign_word(k) & neg))) ^ desc; }
    // Inverse of to_order: once desc is undone, the sign bit of an order word
    // is set exactly for keys that were non-negative.
    __device__ __forceinline__ U from_order(U m) const
    {
        const U a = m ^ desc;
        return a ^ (flip | (~sign_word(a) & neg));
    }
};

// Number of set bits of `mask` in lanes below this lane.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t ballot(bool pred) { return __builtin_amdgcn_ballot_w64(pred); }

// acc & ~(m ^ sel): keep the lanes of `acc` whose ballot bit in `m` equals
// this lane's bit (sel = all ones or zero), as one 3-input bit operation.
// The truth table is indexed by (acc, m, sel) as a 3-bit number; it is true at
// (1,0,0) and (1,1,1).
__device__ __forceinline__ uint32_t keep_equal_bits(uint32_t acc, uint32_t m, uint32_t sel)
{
    return __builtin_amdgcn_bitop3_b32(acc, m, sel, 0x90);
}

// Counts one key per active lane into the digit histograms of several
// passes: hist[p * bins + digit_p(p)] for p = passes - 1 down to 0.  LDS
// atomics of many lanes on one word are executed one after another, so the
// lanes holding lane 0's digit are counted by one add of their number when
// they are many (a whole wave of presorted keys, 90 % zeros of a sparse
// array); the other lanes add 1 each.  The test stops at the first digit
// (most significant first) without such a group: random keys pay for one
// test per key, skewed keys keep the shortcut on every digit that has one.
template <class DigitOf>
__device__ __forceinline__ void lds_count_passes(uint32_t* hist, int bins, int passes, DigitOf&& digit_p)
{
    const uint64_t act = ballot(true);
    bool check = true;  // wave-uniform
#pragma unroll
    for (int p = passes - 1; p >= 0; --p) {
        const uint32_t d = digit_p(p);
        if (check) {
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            const uint64_t same = ballot(d == d0);
            const uint32_t group = (uint32_t)__popcll(same);
            if (group >= 8) {
                if (lanes_below(act) == 0)
                    atomicAdd(&hist[p * bins + (int)d0], group);
                if (d != d0)
                    atomicAdd(&hist[p * bins + (int)d], 1u);
                continue;
            }
            check = false;
        }
        atomicAdd(&hist[p * bins + (int)d], 1u);
    }
}

// Returns x unchanged, but only once y has been computed: an empty asm that
// claims to read y and rewrite x, to order otherwise independent work.
__device__ __forceinline__ uint32_t after(uint32_t x, uint32_t y)
{
    asm volatile("" : "+v"(x) : "v"(y));
    return x;
}

// Returns x unchanged, computed at this point: the compiler may not defer the
// arithmetic that produces x to its first use.  Used where deferring would keep
// the operands of x (several registers) alive instead of x itself.
__device__ __forceinline__ uint32_t materialize(uint32_t x)
{
    asm volatile("" : "+v"(x));
    return x;
}

// Makes a uniform value (a kernel argument) present in scalar registers at
// this point: its load is issued early instead of at its first use.
template <typename T>
__device__ __forceinline__ void in_sgprs(T x)
{
    asm volatile("" ::"s"(x));
}

// base[idx] for a 32-bit index: the byte offset is formed in 32 bits, so the
// load takes one offset register and a base held in scalar registers instead
// of a 64-bit address per element.  Requires idx * sizeof(T) < 2^32.
template <typename T>
__device__ __forceinline__ T load_off32(const T* base, uint32_t idx)
{
    return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + (uint32_t)(idx * (uint32_t)sizeof(T)));
}

// All ones if bit b of x is set, else zero (a sign-extended 1-bit field).
// Written as one instruction so that the compiler tests this value for the
// ballot instead of re-deriving the bit with a shift and a compare.
template <int B>
__device__ __forceinline__ uint32_t bit_mask_of_c(uint32_t x)
{
    uint32_t r;
    asm("v_bfe_i32 %0, %1, %2, 1" : "=v"(r) : "v"(x), "i"(B));
    return r;
}
__device__ __forceinline__ uint32_t bit_mask_of(uint32_t x, int b)
{
    switch (b) {
    case 0: return bit_mask_of_c<0>(x);
    case 1: return bit_mask_of_c<1>(x);
    case 2: return bit_mask_of_c<2>(x);
    case 3: return bit_mask_of_c<3>(x);
    case 4: return bit_mask_of_c<4>(x);
    case 5: return bit_mask_of_c<5>(x);
    case 6: return bit_mask_of_c<6>(x);
    case 7: return bit_mask_of_c<7>(x);
    case 8: return bit_mask_of_c<8>(x);
    case 9: return bit_mask_of_c<9>(x);
    case 10: return bit_mask_of_c<10>(x);
    default: return bit_mask_of_c<11>(x);
    }
}

__device__ __forceinline__ int lane_id() { return (int)__builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Agent-scope relaxed atomics for words that other workgroups (on any XCD)
// poll while this kernel runs.  Flag and payload share one word, so no
// further ordering is needed.
template <typename T>
__device__ __forceinline__ T load_agent(const T* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void store_agent(T* p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Marks a device-side error in a host-visible word (pinned host memory that
// the host polls without synchronizing).  A plain system-scope store of the
// error bit: no atomic crosses to host memory, and every writer stores a
// nonzero value, so any failure leaves the word nonzero.
__device__ __forceinline__ void report_host_error(uint32_t* host_error, uint32_t bit)
{
    if (host_error)
        __hip_atomic_store(host_error, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Exclusive scan of one uint32 per thread across a workgroup of THREADS
// threads.  `wave_tot` must hold THREADS/64 words of LDS.  Returns the
// exclusive prefix and writes the workgroup total to *total.  Contains one
// barrier; the caller must barrier before `wave_tot` is reused.
template <int THREADS>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* wave_tot, uint32_t* total)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        uint32_t y = __shfl_up(x, o, kWave);
        if (lane >= o)
            x += y;
    }
    if (lane == kWave - 1)
        wave_tot[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int i = 0; i < THREADS / kWave; ++i) {
        uint32_t t = wave_tot[i];
        before += (i < w) ? t : 0u;
        all += t;
    }
    *total = all;
    return before + x - v;
}

}  // namespace evosort
