// One-workgroup sort for arrays below the fallback threshold (the branch of
// Sec. 4.3, Algorithm 6 that hands small arrays to the platform's own sort).
//
// One launch of one workgroup: the one-workgroup LSD radix sort (8-bit
// digits; keys, values or indices stay in registers and LDS for every pass),
// with the workgroup shape picked by the array length so that short arrays do
// not pay for the ranks of empty items.  Stable, like every routine here.
#include "block_lsd.hpp"
#include "common.hpp"
#include "small_sort.hpp"

namespace evosort {

namespace {

// Workgroup shapes, smallest first; the last one holds the capacity.  Wave w
// holds keys [w*64*items, (w+1)*64*items), so a shape with few items per
// thread keeps every wave of the workgroup busy on a short array.
struct SmallShape {
    int threads;
    int items;
};
constexpr int kSmallShapeCount = 6;
// 4-byte keys, and 8-byte keys without values
constexpr SmallShape kSmallShapes[kSmallShapeCount] = {{64, 8}, {256, 4}, {256, 8}, {512, 8}, {1024, 8}, {1024, 16}};
// 8-byte keys with values or indices (registers: 16 keys and 16 values per thread need 512 threads)
constexpr SmallShape kSmallShapes8V[kSmallShapeCount] = {{64, 8}, {256, 4}, {256, 8}, {512, 8}, {1024, 8}, {512, 16}};
static_assert(1024 * 16 == kSmallCapacity && 512 * 16 == kSmallCapacity8V, "the largest shape holds the capacity");

// Keys and values share the staging area unless that would not fit in LDS.
template <int KB, int VB, int THREADS, int ITEMS>
constexpr bool split_staging()
{
    return (size_t)THREADS * ITEMS * (KB + VB) > 128 * 1024;
}

template <int KB, int VB, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void small_sort_kernel(SmallSortArgs a, OrderMap<typename KeyWord<KB>::U> om)
{
    constexpr bool SPLIT = split_staging<KB, VB, THREADS, ITEMS>();
    __shared__ BlockLsdLds<KB, VB, THREADS, ITEMS, SPLIT> L;
    const bool argsort = a.mode == SMALL_MODE_ARGSORT;
    if (a.error_word && threadIdx.x == 0)
        *a.error_word = 0;
    const BlockLsdIo io{a.keys_in, a.keys_out, a.vals_in, a.vals_out, argsort, argsort};
    block_lsd_sort<KB, VB, THREADS, ITEMS, SPLIT>(io, om, L, 0, (uint32_t)a.n);
}

template <int KB, int VB, int THREADS, int ITEMS>
hipError_t launch_shape(const KeyDesc& kd, const SmallSortArgs& a, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    static_assert(sizeof(BlockLsdLds<KB, VB, THREADS, ITEMS, split_staging<KB, VB, THREADS, ITEMS>()>) <=
                      160 * 1024,
                  "one workgroup fits in one CU's LDS");
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL((small_sort_kernel<KB, VB, THREADS, ITEMS>), dim3(1), dim3(THREADS), 0, s, a, om);
    return hipGetLastError();
}

// The first shape, from index I on, that holds n keys.
template <int KB, int VB, int I>
hipError_t launch_t(const KeyDesc& kd, const SmallSortArgs& a, hipStream_t s)
{
    constexpr SmallShape sh = KB == 8 && VB != 0 ? kSmallShapes8V[I] : kSmallShapes[I];
    if constexpr (I + 1 < kSmallShapeCount) {
        if (a.n > (int64_t)sh.threads * sh.items)
            return launch_t<KB, VB, I + 1>(kd, a, s);
    }
    return launch_shape<KB, VB, sh.threads, sh.items>(kd, a, s);
}

}  // namespace

int64_t small_sort_capacity(int key_bytes, int val_bytes)
{
    return key_bytes == 8 && val_bytes != 0 ? kSmallCapacity8V : kSmallCapacity;
}

hipError_t launch_small_sort(const KeyDesc& kd, int val_bytes, const SmallSortArgs& a, hipStream_t s)
{
    if (a.n < 0 || a.n > small_sort_capacity(kd.bytes, val_bytes))
        return hipErrorInvalidValue;
    if (a.n == 0)
        return hipSuccess;
    if (kd.bytes == 4) {
        if (val_bytes == 0)
            return launch_t<4, 0, 0>(kd, a, s);
        if (val_bytes == 4)
            return launch_t<4, 4, 0>(kd, a, s);
        return launch_t<4, 8, 0>(kd, a, s);
    }
    if (val_bytes == 0)
        return launch_t<8, 0, 0>(kd, a, s);
    if (val_bytes == 4)
        return launch_t<8, 4, 0>(kd, a, s);
    return launch_t<8, 8, 0>(kd, a, s);
}

}  // namespace evosort
