// Device-side planning of the batched segmented sort: classification of the
// segments, and digit histograms and bases of the large ones.
#include "common.hpp"
#include "segmented.hpp"

namespace evosort {

hipError_t seg_block_dispatch_k4_v0(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);
hipError_t seg_block_dispatch_k4_v4(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);
hipError_t seg_block_dispatch_k4_v8(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);
hipError_t seg_block_dispatch_k8_v0(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);
hipError_t seg_block_dispatch_k8_v4(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);
hipError_t seg_block_dispatch_k8_v8(int, const KeyDesc&, const SegBlockArgs&, uint32_t, hipStream_t);

namespace {

constexpr int kSegThreads = 256;  // = kSegBins: one digit per thread in the scan

// Index of this lane's item in a list whose length is *counter, for the lanes
// with `mine` set; one atomic per wave.  Every lane of the wave must call it.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, bool mine)
{
    const uint64_t m = ballot(mine);
    if (m == 0)
        return 0;
    const int leader = __builtin_ctzll(m);
    uint32_t base = 0;
    if (lane_id() == leader)
        base = atomicAdd(counter, (uint32_t)__popcll(m));
    base = __shfl(base, leader, kWave);
    return base + lanes_below(m);
}

// Exclusive sum of x over the lanes of the wave; *total gets the wave's sum.
__device__ __forceinline__ uint32_t wave_exclusive_sum(uint32_t x, uint32_t* total)
{
    const int lane = lane_id();
    uint32_t v = x;
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        const uint32_t y = __shfl_up(v, o, kWave);
        if (lane >= o)
            v += y;
    }
    *total = __shfl(v, kWave - 1, kWave);
    return v - x;
}

// One thread per offset: offsets must be non-decreasing within [0, n] and
// every segment shorter than 2^30 keys.  Any violation sets the error word,
// and the classification that follows then takes no segment at all, so the
// bounds the scratch is sized for (segments disjoint inside [0, n)) hold for
// every segment that is sorted.
__global__ __launch_bounds__(kSegThreads) void seg_validate_kernel(SegClassifyArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * kSegThreads + threadIdx.x;
    if (i > a.nseg)
        return;
    const int64_t x = a.offsets[i];
    bool bad = x < 0 || x > a.n;
    if (i < a.nseg) {
        const int64_t y = a.offsets[i + 1];
        bad = bad || y < x || y - x >= ((int64_t)1 << 30);
    }
    if (bad) {
        atomicOr(a.error_word, kDeviceErrBadSegment);
        report_host_error(a.host_error, kDeviceErrBadSegment);
    }
}

// One thread per segment.
__global__ __launch_bounds__(kSegThreads) void seg_classify_kernel(SegClassifyArgs a)
{
    const int64_t s = (int64_t)blockIdx.x * kSegThreads + threadIdx.x;
    if (*a.error_word & kDeviceErrBadSegment)
        return;  // uniform: the validation launch has finished
    int cls = -1;
    int64_t begin = 0;
    uint32_t len = 0, ntiles = 0;
    if (s < a.nseg) {
        begin = a.offsets[s];
        len = (uint32_t)(a.offsets[s + 1] - begin);
        if (len > 0) {
            if ((int64_t)len < a.block_limit) {
                cls = a.classes - 1;  // smallest class that holds the segment
                for (int c = a.classes - 2; c >= 0; --c)
                    if ((int64_t)len <= a.cap[c])
                        cls = c;
            } else {
                cls = a.classes;  // large
                ntiles = (len + a.tile_keys - 1) / a.tile_keys;
            }
        }
    }
    for (int c = 0; c < a.classes; ++c) {
        const uint32_t idx = wave_append(&a.ctr->class_count[c], cls == c);
        if (cls == c)
            a.lists[(size_t)c * a.nseg + idx] = (uint32_t)s;
    }
    // Large segments: a slot, and a contiguous range of tiles.
    const bool big = cls == a.classes;
    const uint32_t slot = wave_append(&a.ctr->class_count[kSegMaxClasses], big);
    uint32_t total;
    const uint32_t excl = wave_exclusive_sum(ntiles, &total);
    uint32_t tbase = 0;
    if (total) {
        if (lane_id() == 0)
            tbase = atomicAdd(&a.ctr->tile_count, total);
        tbase = __shfl(tbase, 0, kWave);
    }
    if (big) {
        a.lists[(size_t)a.classes * a.nseg + slot] = (uint32_t)s;
        a.large[slot] = SegLarge{begin, len, tbase + excl};
    }
}

// Per large segment: zero its histogram and write its entries of the tile ->
// segment map.
__global__ __launch_bounds__(kSegThreads) void seg_setup_kernel(SegLargeArgs a, uint32_t tile_keys)
{
    const uint32_t nlarge = *a.nlarge;
    const int words = a.passes * kSegBins;
    for (uint32_t j = blockIdx.x; j < nlarge; j += gridDim.x) {
        const SegLarge g = a.large[j];
        for (int i = threadIdx.x; i < words; i += kSegThreads)
            a.hist[(size_t)j * words + i] = 0;
        const uint32_t ntiles = (g.len + tile_keys - 1) / tile_keys;
        for (uint32_t i = threadIdx.x; i < ntiles; i += kSegThreads)
            a.tile_slot[g.first_tile + i] = j;
    }
}

// Digit histograms of the large segments.  Workgroup g takes tiles
// [g*group, g*group + group) and keeps one set of LDS counters per wave while
// consecutive tiles belong to one segment.  A segment whose tiles all lie in
// this range is stored directly; otherwise the counts are added atomically.
// Each tile's look-back words of every pass are zeroed here.
template <int KB>
__global__ __launch_bounds__(kSegThreads) void seg_histogram_kernel(SegHistArgs a,
                                                                    OrderMap<typename KeyWord<KB>::U> om)
{
    using U = typename KeyWord<KB>::U;
    constexpr int PASSES = KB;  // 8-bit digits
    constexpr int WAVES = kSegThreads / kWave;
    constexpr int WORDS = PASSES * kSegBins;
    __shared__ uint32_t h[WAVES][WORDS];

    const uint32_t count = *a.tile_count;
    const uint32_t t0 = blockIdx.x * a.group;
    if (t0 >= count)
        return;
    const uint32_t t1 = t0 + a.group < count ? t0 + a.group : count;

    auto zero = [&] {
        for (int i = threadIdx.x; i < WAVES * WORDS; i += kSegThreads)
            (&h[0][0])[i] = 0;
    };
    auto flush = [&](uint32_t slot, const SegLarge& g) {
        const uint32_t nt = (g.len + a.tile_keys - 1) / a.tile_keys;
        const bool whole = g.first_tile >= t0 && g.first_tile + nt <= t1;
        uint32_t* dst = a.hist + (size_t)slot * WORDS;
        for (int i = threadIdx.x; i < WORDS; i += kSegThreads) {
            uint32_t v = 0;
#pragma unroll
            for (int w = 0; w < WAVES; ++w)
                v += h[w][i];
            if (whole)
                dst[i] = v;
            else if (v)
                atomicAdd(&dst[i], v);
        }
    };

    uint32_t* mine = h[threadIdx.x / kWave];
    auto count_key = [&](U k) {
        const U u = om.to_order(k);
        lds_count_passes(mine, kSegBins, PASSES,
                         [&](int p) { return (uint32_t)((u >> (p * kSegBits)) & (U)(kSegBins - 1)); });
    };

    zero();
    __syncthreads();
    uint32_t cur = a.tile_slot[t0];
    SegLarge g = a.large[cur];
    const U* keys = reinterpret_cast<const U*>(a.keys);
    for (uint32_t t = t0; t < t1; ++t) {
        const uint32_t slot = a.tile_slot[t];
        if (slot != cur) {
            __syncthreads();
            flush(cur, g);
            __syncthreads();
            zero();
            __syncthreads();
            cur = slot;
            g = a.large[slot];
        }
#pragma unroll
        for (int p = 0; p < PASSES; ++p)
            a.status[(size_t)p * a.status_pass_words + (size_t)t * kSegBins + threadIdx.x] = 0;

        const uint32_t lt = t - g.first_tile;
        const uint32_t done = lt * a.tile_keys;
        const uint32_t cnt = g.len - done < a.tile_keys ? g.len - done : a.tile_keys;
        const U* kp = keys + g.begin + done;
        // scalar head up to 16-byte alignment, 16-byte body, scalar tail
        constexpr int VEC = 16 / KB;
        uint32_t head = (uint32_t)(((16 - (reinterpret_cast<uintptr_t>(kp) & 15)) & 15) / KB);
        if (head > cnt)
            head = cnt;
        if (threadIdx.x < head)
            count_key(kp[threadIdx.x]);
        const uint4* kv = reinterpret_cast<const uint4*>(kp + head);
        const uint32_t nvec = (cnt - head) / VEC;
        constexpr int UNROLL = 4;
        uint32_t v = threadIdx.x;
        for (; v + (UNROLL - 1) * kSegThreads < nvec; v += UNROLL * kSegThreads) {
            uint4 w[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                w[u] = kv[v + u * kSegThreads];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                U k[VEC];
                __builtin_memcpy(k, &w[u], 16);
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    count_key(k[j]);
            }
        }
        for (; v < nvec; v += kSegThreads) {
            const uint4 w = kv[v];
            U k[VEC];
            __builtin_memcpy(k, &w, 16);
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                count_key(k[j]);
        }
        for (uint32_t i = head + nvec * VEC + threadIdx.x; i < cnt; i += kSegThreads)
            count_key(kp[i]);
    }
    __syncthreads();
    flush(cur, g);
}

// Digit bases of each large segment and pass: exclusive prefix sums of its
// counts (positions relative to the segment's first key).
__global__ __launch_bounds__(kSegThreads) void seg_scan_kernel(SegLargeArgs a)
{
    __shared__ uint32_t wtot[kSegThreads / kWave];
    const uint32_t nlarge = *a.nlarge;
    const int words = a.passes * kSegBins;
    for (uint32_t j = blockIdx.x; j < nlarge; j += gridDim.x) {
        for (int p = 0; p < a.passes; ++p) {
            const size_t i = (size_t)j * words + (size_t)p * kSegBins + threadIdx.x;
            uint32_t total;
            const uint32_t excl = block_exclusive_scan<kSegThreads>(a.hist[i], wtot, &total);
            a.bases[i] = excl;
            __syncthreads();  // wtot is reused by the next scan
        }
    }
}

}  // namespace

hipError_t launch_seg_classify(const SegClassifyArgs& a, hipStream_t s)
{
    if (a.nseg <= 0)
        return hipSuccess;
    const int64_t vgrid = (a.nseg + 1 + kSegThreads - 1) / kSegThreads;
    hipLaunchKernelGGL(seg_validate_kernel, dim3((uint32_t)vgrid), dim3(kSegThreads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    const int64_t grid = (a.nseg + kSegThreads - 1) / kSegThreads;
    hipLaunchKernelGGL(seg_classify_kernel, dim3((uint32_t)grid), dim3(kSegThreads), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_seg_setup(const SegLargeArgs& a, uint32_t tile_keys, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL(seg_setup_kernel, dim3(grid), dim3(kSegThreads), 0, s, a, tile_keys);
    return hipGetLastError();
}

hipError_t launch_seg_histogram(const KeyDesc& kd, const SegHistArgs& a, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    if (kd.bytes == 4) {
        OrderMap<uint32_t> om{(uint32_t)kd.flip, (uint32_t)kd.neg, (uint32_t)kd.desc};
        hipLaunchKernelGGL(seg_histogram_kernel<4>, dim3(grid), dim3(kSegThreads), 0, s, a, om);
    } else {
        OrderMap<uint64_t> om{kd.flip, kd.neg, kd.desc};
        hipLaunchKernelGGL(seg_histogram_kernel<8>, dim3(grid), dim3(kSegThreads), 0, s, a, om);
    }
    return hipGetLastError();
}

hipError_t launch_seg_block_sort(const KeyDesc& kd, int val_bytes, int cls, const SegBlockArgs& a,
                                 uint32_t max_grid, hipStream_t s)
{
    if (kd.bytes == 4) {
        if (val_bytes == 0)
            return seg_block_dispatch_k4_v0(cls, kd, a, max_grid, s);
        if (val_bytes == 4)
            return seg_block_dispatch_k4_v4(cls, kd, a, max_grid, s);
        return seg_block_dispatch_k4_v8(cls, kd, a, max_grid, s);
    }
    if (val_bytes == 0)
        return seg_block_dispatch_k8_v0(cls, kd, a, max_grid, s);
    if (val_bytes == 4)
        return seg_block_dispatch_k8_v4(cls, kd, a, max_grid, s);
    return seg_block_dispatch_k8_v8(cls, kd, a, max_grid, s);
}

hipError_t launch_seg_scan(const SegLargeArgs& a, uint32_t grid, hipStream_t s)
{
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL(seg_scan_kernel, dim3(grid), dim3(kSegThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace evosort
