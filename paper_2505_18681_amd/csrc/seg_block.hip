// One-workgroup sort of the small segments of a batched segmented sort.
//
// A persistent workgroup takes segments from its class's list (an atomic
// ticket) and sorts each one entirely inside the CU with the one-workgroup
// LSD sort (keys and values stay in registers and LDS for all 8-bit passes,
// so HBM sees one read and one write per key).
//
// Compiled once per (key bytes, value bytes) pair with -DEVOSORT_KB/-DEVOSORT_VB.
#include "block_lsd.hpp"
#include "common.hpp"
#include "segmented.hpp"

#ifndef EVOSORT_KB
#error "EVOSORT_KB must be defined"
#endif
#ifndef EVOSORT_VB
#error "EVOSORT_VB must be defined"
#endif

#define EVOSORT_CAT4(a, b, c, d) a##b##c##d
#define EVOSORT_XCAT4(a, b, c, d) EVOSORT_CAT4(a, b, c, d)
#define EVOSORT_NAME(kb, vb) EVOSORT_XCAT4(seg_block_dispatch_k, kb, _v, vb)

namespace evosort {

static_assert(kSegBits == kBlockLsdBits, "segments are sorted with the segmented routine's digit width");

namespace {

template <int KB, int VB, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void seg_block_sort_kernel(SegBlockArgs a,
                                                                 OrderMap<typename KeyWord<KB>::U> om)
{
    __shared__ BlockLsdLds<KB, VB, THREADS, ITEMS, false> L;
    const BlockLsdIo io{a.keys_in, a.keys_out, a.vals_in, a.vals_out, false, false};
    const uint32_t count = *a.count;
    for (;;) {
        if (threadIdx.x == 0)
            L.job = atomicAdd(a.ticket, 1u);
        __syncthreads();
        const uint32_t j = L.job;
        if (j >= count)
            break;  // uniform across the workgroup
        const uint32_t seg = a.list[j];
        const int64_t begin = a.offsets[seg];
        const uint32_t len = (uint32_t)(a.offsets[seg + 1] - begin);
        // block_lsd_sort ends with a barrier, so every thread has read L.job
        // before thread 0 overwrites it
        block_lsd_sort<KB, VB, THREADS, ITEMS, false>(io, om, L, begin, len);
    }
}

template <int CLS>
hipError_t launch_class(const KeyDesc& kd, const SegBlockArgs& a, uint32_t max_grid, hipStream_t s)
{
    constexpr int RB = EVOSORT_KB + EVOSORT_VB;
    constexpr SegClass c = seg_class(RB, CLS);
    using U = typename KeyWord<EVOSORT_KB>::U;
    static_assert(sizeof(BlockLsdLds<EVOSORT_KB, EVOSORT_VB, c.threads, c.items, false>) <= 80 * 1024,
                  "two workgroups of a class fit in one CU's LDS");
    auto kernel = seg_block_sort_kernel<EVOSORT_KB, EVOSORT_VB, c.threads, c.items>;
    static int resident = 0;  // one per instantiation
    if (resident == 0) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, c.threads, 0) == hipSuccess && cus > 0 &&
            per_cu > 0)
            resident = cus * per_cu;
        else {
            (void)hipGetLastError();
            resident = 1024;  // any grid is correct; this only sizes the persistent launch
        }
    }
    const uint32_t grid = max_grid < (uint32_t)resident ? max_grid : (uint32_t)resident;
    if (grid == 0)
        return hipSuccess;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL(kernel, dim3(grid), dim3(c.threads), 0, s, a, om);
    return hipGetLastError();
}

}  // namespace

hipError_t EVOSORT_NAME(EVOSORT_KB, EVOSORT_VB)(int cls, const KeyDesc& kd, const SegBlockArgs& a,
                                                 uint32_t max_grid, hipStream_t s)
{
    constexpr int classes = seg_class_count(EVOSORT_KB + EVOSORT_VB);
    switch (cls) {
    case 0:
        return launch_class<0>(kd, a, max_grid, s);
    case 1:
        return launch_class<1>(kd, a, max_grid, s);
    case 2:
        return launch_class<2>(kd, a, max_grid, s);
    case 3:
        if constexpr (classes > 3)
            return launch_class<3>(kd, a, max_grid, s);
        return hipErrorInvalidValue;
    default:
        return hipErrorInvalidValue;
    }
}

}  // namespace evosort
