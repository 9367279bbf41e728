// One-workgroup sort of the small segments of a batched segmented sort.
//
// A persistent workgroup takes segments from its class's list (an atomic
// ticket) and sorts each one entirely inside the CU: the keys (and values)
// stay in registers and LDS for all 8-bit LSD passes, so HBM sees one read and
// one write per key.  Each pass ranks the keys stably with the same wave64
// lane-bucket rank as the device-wide pass (Sec. 4, Algorithms 4 and 5 at
// workgroup scale: per-digit counts, prefix sums, placement), then scatters
// them through LDS and reads them back in the striped order the next pass
// ranks in.
//
// Compiled once per (key bytes, value bytes) pair with -DEVOSORT_KB/-DEVOSORT_VB.
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

namespace {

template <int KB, int VB, int THREADS, int ITEMS>
struct BlockLds {
    static constexpr int WAVES = THREADS / kWave;
    static constexpr int CAP = THREADS * ITEMS;
    // counters [WAVES][256] uint32 and lane buckets [WAVES][256] uint64,
    // sharing storage with the staging area of one pass's scatter
    static constexpr size_t BUCKET_OFFSET = ((size_t)WAVES * kSegBins * 4 + 15) & ~(size_t)15;
    static constexpr size_t HIST_BYTES = BUCKET_OFFSET + (size_t)WAVES * kSegBins * 8;
    static constexpr size_t STAGE_BYTES = (size_t)CAP * KB + (size_t)(VB ? CAP * VB : 0);
    static constexpr size_t UNION_BYTES = HIST_BYTES > STAGE_BYTES ? HIST_BYTES : STAGE_BYTES;
    __attribute__((aligned(16))) unsigned char uni[UNION_BYTES];
    uint32_t wtot[WAVES];
    uint32_t job;
};

// Sorts keys [begin, begin + len) (len <= THREADS * ITEMS).  Wave w holds
// positions [w*64*ITEMS, (w+1)*64*ITEMS), item i lane-striped (position
// w*64*ITEMS + i*64 + lane), so ranking items in order and lanes in order
// visits positions in order: each pass is stable.
template <int KB, int VB, int THREADS, int ITEMS>
__device__ __forceinline__ void sort_segment(const SegBlockArgs& a, const OrderMap<typename KeyWord<KB>::U>& om,
                                             BlockLds<KB, VB, THREADS, ITEMS>& L, int64_t begin, uint32_t len)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using Lds = BlockLds<KB, VB, THREADS, ITEMS>;
    constexpr int PASSES = KB;  // 8-bit digits
    constexpr int BINS = kSegBins;
    constexpr int WAVES = Lds::WAVES;
    constexpr int CAP = Lds::CAP;
    constexpr int WAVE_KEYS = kWave * ITEMS;
    constexpr int BPT = (BINS + THREADS - 1) / THREADS;

    uint32_t* s_whist = reinterpret_cast<uint32_t*>(L.uni);
    uint64_t* s_bkt = reinterpret_cast<uint64_t*>(L.uni + Lds::BUCKET_OFFSET);
    U* s_keys = reinterpret_cast<U*>(L.uni);
    V* s_vals = reinterpret_cast<V*>(L.uni + (size_t)CAP * KB);

    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const uint32_t off0 = (uint32_t)(w * WAVE_KEYS + lane);
    const uint32_t wave_base = (uint32_t)(w * WAVE_KEYS);

    U k[ITEMS];
    V v[VB ? ITEMS : 1];
    {
        const U* kin = reinterpret_cast<const U*>(a.keys_in) + begin;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t q = off0 + (uint32_t)(i * kWave);
            k[i] = q < len ? kin[q] : (U)0;
        }
        if constexpr (VB != 0) {
            const V* vin = reinterpret_cast<const V*>(a.vals_in) + begin;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t q = off0 + (uint32_t)(i * kWave);
                v[i] = q < len ? vin[q] : (V)0;
            }
        }
    }

    const uint64_t my_bit = 1ull << lane;
    for (int p = 0; p < PASSES; ++p) {
        const int shift = p * kSegBits;
        for (int i = threadIdx.x; i < WAVES * BINS; i += THREADS) {
            s_whist[i] = 0;
            s_bkt[i] = 0;
        }
        __syncthreads();

        // stable rank inside each wave (lane buckets, as in the device-wide pass)
        uint32_t* wh = s_whist + w * BINS;
        uint64_t* bkt = s_bkt + w * BINS;
        uint32_t rk[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            rk[i] = 0;
            if (wave_base + (uint32_t)(i * kWave) < len) {  // uniform across the wave
                const uint32_t d = (uint32_t)((om.to_order(k[i]) >> shift) & (U)(BINS - 1));
                const bool valid = off0 + (uint32_t)(i * kWave) < len;
                // lane 0's digit group from one ballot, the others through the buckets
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                const uint64_t same = ballot(d == d0);
                const uint64_t vmask = ballot(valid);
                if (same != ~0ull && d != d0 && valid)
                    atomicOr(reinterpret_cast<unsigned long long*>(&bkt[d]), (unsigned long long)my_bit);
                const uint64_t peers = d == d0 ? (same & vmask) : bkt[d];
                const uint32_t old = wh[d];
                const uint32_t below = lanes_below(peers);
                if (valid && below == 0) {
                    bkt[d] = 0;
                    wh[d] = old + (uint32_t)__popcll(peers);
                }
                rk[i] = (d << 16) | (old + below);
            }
        }
        __syncthreads();

        // digit totals, their prefix sums, and each wave's first position per digit
        uint32_t cnt[BPT];
        uint32_t tsum = 0;
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = threadIdx.x * BPT + j;
            uint32_t c = 0;
            if (b < BINS) {
#pragma unroll
                for (int ww = 0; ww < WAVES; ++ww)
                    c += s_whist[ww * BINS + b];
            }
            cnt[j] = c;
            tsum += c;
        }
        uint32_t total;
        uint32_t run = block_exclusive_scan<THREADS>(tsum, L.wtot, &total);
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = threadIdx.x * BPT + j;
            if (b < BINS) {
                uint32_t r = run;
#pragma unroll
                for (int ww = 0; ww < WAVES; ++ww) {
                    const uint32_t c = s_whist[ww * BINS + b];
                    s_whist[ww * BINS + b] = r;
                    r += c;
                }
            }
            run += cnt[j];
        }
        __syncthreads();

#pragma unroll
        for (int i = 0; i < ITEMS; ++i)
            rk[i] = off0 + (uint32_t)(i * kWave) < len ? s_whist[w * BINS + (rk[i] >> 16)] + (rk[i] & 0xffffu)
                                                       : 0xffffffffu;
        __syncthreads();  // counters are dead: the staging area may be written
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (rk[i] != 0xffffffffu) {
                s_keys[rk[i]] = k[i];
                if constexpr (VB != 0)
                    s_vals[rk[i]] = v[i];
            }
        }
        __syncthreads();

        if (p == PASSES - 1) {
            U* kout = reinterpret_cast<U*>(a.keys_out) + begin;
            for (uint32_t q = threadIdx.x; q < len; q += THREADS)
                kout[q] = s_keys[q];
            if constexpr (VB != 0) {
                V* vout = reinterpret_cast<V*>(a.vals_out) + begin;
                for (uint32_t q = threadIdx.x; q < len; q += THREADS)
                    vout[q] = s_vals[q];
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t q = off0 + (uint32_t)(i * kWave);
                if (q < len) {
                    k[i] = s_keys[q];
                    if constexpr (VB != 0)
                        v[i] = s_vals[q];
                }
            }
        }
        __syncthreads();  // staging reads are done before the counters reuse it
    }
}

template <int KB, int VB, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void seg_block_sort_kernel(SegBlockArgs a,
                                                                 OrderMap<typename KeyWord<KB>::U> om)
{
    __shared__ BlockLds<KB, VB, THREADS, ITEMS> L;
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
        // sort_segment ends with a barrier, so every thread has read L.job
        // before thread 0 overwrites it
        sort_segment<KB, VB, THREADS, ITEMS>(a, om, L, begin, len);
    }
}

template <int CLS>
hipError_t launch_class(const KeyDesc& kd, const SegBlockArgs& a, uint32_t max_grid, hipStream_t s)
{
    constexpr int RB = EVOSORT_KB + EVOSORT_VB;
    constexpr SegClass c = seg_class(RB, CLS);
    using U = typename KeyWord<EVOSORT_KB>::U;
    static_assert(sizeof(BlockLds<EVOSORT_KB, EVOSORT_VB, c.threads, c.items>) <= 80 * 1024,
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
