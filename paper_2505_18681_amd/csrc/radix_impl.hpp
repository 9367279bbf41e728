// Block-based LSD radix sort kernels for gfx950 (Sec. 4, Algorithms 4 and 5,
// re-designed for one GPU):
//
//   radix_histogram_kernel  one read of the keys fills the digit histogram of
//                           every pass (the paper recounts before each pass;
//                           the count of a digit position does not depend on
//                           the order the keys are in, so one read suffices);
//   radix_scan_kernel       exclusive prefix sums of each pass's histogram:
//                           the first output slot of every digit;
//   radix_pass_kernel       one pass: rank a tile of keys stably by digit
//                           inside the workgroup, find the tile's offset within
//                           each digit's output range by a chained scan over
//                           tiles (decoupled look-back), then write the tile
//                           through LDS so that keys of one digit leave as one
//                           contiguous run.
#pragma once

#include "common.hpp"
#include "kernels.hpp"
#include "segmented.hpp"

namespace evosort {

// ------------------------------------------------------------------------
// All-pass histogram
// ------------------------------------------------------------------------
// LDS holds `copies` private histograms (passes << bits words each); wave w
// counts into copy w % copies, which spreads LDS atomic traffic when many keys
// share a digit.  Counts are flushed to the global uint64 histogram once.
template <int KB, int THREADS>
__global__ __launch_bounds__(THREADS) void radix_histogram_kernel(const typename KeyWord<KB>::U* __restrict__ keys,
                                                                  int64_t n, OrderMap<typename KeyWord<KB>::U> om,
                                                                  int bits, int pass0, int passes, int copies,
                                                                  unsigned long long* __restrict__ hist)
{
    using U = typename KeyWord<KB>::U;
    extern __shared__ uint32_t lds_hist[];
    const int bins = 1 << bits;
    const int per_copy = passes * bins;
    for (int i = threadIdx.x; i < copies * per_copy; i += THREADS)
        lds_hist[i] = 0;
    __syncthreads();

    uint32_t* mine = lds_hist + (int)((threadIdx.x / kWave) % copies) * per_copy;
    const U mask = (U)(bins - 1);
    auto count = [&](U k) {
        const U u = om.to_order(k);
        for (int p = 0; p < passes; ++p)
            atomicAdd(&mine[p * bins + (int)((u >> ((pass0 + p) * bits)) & mask)], 1u);
    };

    constexpr int VEC = 16 / KB;  // keys per 16-byte load
    constexpr int UNROLL = 4;     // 16-byte loads in flight per thread
    const int64_t stride = (int64_t)gridDim.x * THREADS;
    const int64_t gtid = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(keys) & 15) == 0) {
        const int64_t nvec = n / VEC;
        const uint4* kv = reinterpret_cast<const uint4*>(keys);
        int64_t v = gtid;
        // Issue UNROLL independent loads before counting any of them.
        for (; v + (UNROLL - 1) * stride < nvec; v += UNROLL * stride) {
            uint4 w[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                w[u] = kv[v + u * stride];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                U k[VEC];
                __builtin_memcpy(k, &w[u], 16);
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    count(k[j]);
            }
        }
        for (; v < nvec; v += stride) {
            uint4 w = kv[v];
            U k[VEC];
            __builtin_memcpy(k, &w, 16);
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                count(k[j]);
        }
        done = nvec * VEC;
    }
    for (int64_t i = done + gtid; i < n; i += stride)
        count(keys[i]);
    __syncthreads();

    for (int i = threadIdx.x; i < per_copy; i += THREADS) {
        uint32_t s = 0;
        for (int c = 0; c < copies; ++c)
            s += lds_hist[c * per_copy + i];
        if (s)
            atomicAdd(&hist[(size_t)pass0 * bins + i], (unsigned long long)s);
    }
}

// The same for 8-bit digits and all passes in one launch (the common case),
// with the pass count known at compile time.  Skewed, presorted and sparse
// keys: lds_count_passes lets one lane count the lanes that share lane 0's
// digit when they are many.
template <int KB, int THREADS, int PASSES>
__global__ __launch_bounds__(THREADS) void radix_histogram8_kernel(const typename KeyWord<KB>::U* __restrict__ keys,
                                                                   int64_t n, OrderMap<typename KeyWord<KB>::U> om,
                                                                   int copies, unsigned long long* __restrict__ hist)
{
    using U = typename KeyWord<KB>::U;
    constexpr int BINS = 256;
    constexpr int PER_COPY = PASSES * BINS;
    extern __shared__ uint32_t lds_hist[];
    for (int i = threadIdx.x; i < copies * PER_COPY; i += THREADS)
        lds_hist[i] = 0;
    __syncthreads();

    uint32_t* mine = lds_hist + (int)((threadIdx.x / kWave) % copies) * PER_COPY;
    auto count = [&](U k) {
        const U u = om.to_order(k);
        lds_count_passes(mine, BINS, PASSES, [&](int p) { return (uint32_t)(u >> (8 * p)) & 0xffu; });
    };

    constexpr int VEC = 16 / KB;
    constexpr int UNROLL = 4;
    const int64_t stride = (int64_t)gridDim.x * THREADS;
    const int64_t gtid = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(keys) & 15) == 0) {
        const int64_t nvec = n / VEC;
        const uint4* kv = reinterpret_cast<const uint4*>(keys);
        int64_t v = gtid;
        for (; v + (UNROLL - 1) * stride < nvec; v += UNROLL * stride) {
            uint4 w[UNROLL];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u)
                w[u] = kv[v + u * stride];
#pragma unroll
            for (int u = 0; u < UNROLL; ++u) {
                U k[VEC];
                __builtin_memcpy(k, &w[u], 16);
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    count(k[j]);
            }
        }
        for (; v < nvec; v += stride) {
            uint4 w = kv[v];
            U k[VEC];
            __builtin_memcpy(k, &w, 16);
#pragma unroll
            for (int j = 0; j < VEC; ++j)
                count(k[j]);
        }
        done = nvec * VEC;
    }
    for (int64_t i = done + gtid; i < n; i += stride)
        count(keys[i]);
    __syncthreads();

    for (int i = threadIdx.x; i < PER_COPY; i += THREADS) {
        uint32_t s = 0;
        for (int c = 0; c < copies; ++c)
            s += lds_hist[c * PER_COPY + i];
        if (s)
            atomicAdd(&hist[i], (unsigned long long)s);
    }
}

// The all-pass histogram once more, walking the keys tile by tile (the radix
// pass's tiles of tile_keys keys): passes 1.. are counted as above, while
// pass 0's digits are counted per tile and written to counts[tile][256].
// With these counts pass 0 knows every tile's output offsets before it starts
// (an exclusive scan over tiles, launch_tile_prefix) and needs no look-back:
// the digit counts of pass 0 depend only on the input order, which is known
// here; those of later passes depend on the previous pass's output.
template <int KB, int THREADS, int PASSES, typename ST>
__global__ __launch_bounds__(THREADS) void radix_histogram8_tiles_kernel(
    const typename KeyWord<KB>::U* __restrict__ keys, int64_t n, OrderMap<typename KeyWord<KB>::U> om, int copies,
    unsigned long long* __restrict__ hist, ST* __restrict__ counts, uint32_t tile_keys, uint32_t tiles)
{
    using U = typename KeyWord<KB>::U;
    constexpr int BINS = 256;
    constexpr int PER_COPY = PASSES * BINS;
    extern __shared__ uint32_t lds_hist[];  // copies * PER_COPY, then the tile's pass-0 row
    uint32_t* tile_row = lds_hist + copies * PER_COPY;
    for (int i = threadIdx.x; i < copies * PER_COPY + BINS; i += THREADS)
        lds_hist[i] = 0;
    __syncthreads();

    uint32_t* mine = lds_hist + (int)((threadIdx.x / kWave) % copies) * PER_COPY;
    // as lds_count_passes, with pass 0 counted into the tile's row
    auto count = [&](U k) {
        const U u = om.to_order(k);
        const uint64_t act = ballot(true);
        bool check = true;  // wave-uniform
#pragma unroll
        for (int p = PASSES - 1; p >= 0; --p) {
            uint32_t* row = p == 0 ? tile_row : mine + p * BINS;
            const uint32_t d = (uint32_t)(u >> (8 * p)) & 0xffu;
            if (check) {
                const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
                const uint64_t same = ballot(d == d0);
                const uint32_t group = (uint32_t)__popcll(same);
                if (group >= 8) {
                    if (lanes_below(act) == 0)
                        atomicAdd(&row[d0], group);
                    if (d != d0)
                        atomicAdd(&row[d], 1u);
                    continue;
                }
                check = false;
            }
            atomicAdd(&row[d], 1u);
        }
    };

    constexpr int VEC = 16 / KB;
    constexpr int UNROLL = 4;
    const bool aligned = (reinterpret_cast<uintptr_t>(keys) & 15) == 0 && (tile_keys % VEC) == 0;
    for (uint32_t t = blockIdx.x; t < tiles; t += gridDim.x) {
        const int64_t start = (int64_t)t * tile_keys;
        const int64_t len = n - start < (int64_t)tile_keys ? n - start : (int64_t)tile_keys;
        const U* tk = keys + start;
        int64_t done = 0;
        if (aligned) {
            const int64_t nvec = len / VEC;
            const uint4* kv = reinterpret_cast<const uint4*>(tk);
            int64_t v = threadIdx.x;
            for (; v + (UNROLL - 1) * THREADS < nvec; v += UNROLL * THREADS) {
                uint4 w[UNROLL];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u)
                    w[u] = kv[v + u * THREADS];
#pragma unroll
                for (int u = 0; u < UNROLL; ++u) {
                    U k[VEC];
                    __builtin_memcpy(k, &w[u], 16);
#pragma unroll
                    for (int j = 0; j < VEC; ++j)
                        count(k[j]);
                }
            }
            for (; v < nvec; v += THREADS) {
                uint4 w = kv[v];
                U k[VEC];
                __builtin_memcpy(k, &w, 16);
#pragma unroll
                for (int j = 0; j < VEC; ++j)
                    count(k[j]);
            }
            done = nvec * VEC;
        }
        for (int64_t i = done + threadIdx.x; i < len; i += THREADS)
            count(tk[i]);
        __syncthreads();
        // the tile's pass-0 counts go out and into the pass-0 row of copy 0
        for (int b = threadIdx.x; b < BINS; b += THREADS) {
            const uint32_t c = tile_row[b];
            counts[(size_t)t * BINS + b] = (ST)c;
            lds_hist[b] += c;
            tile_row[b] = 0;
        }
        __syncthreads();
    }

    for (int i = threadIdx.x; i < PER_COPY; i += THREADS) {
        uint32_t s = 0;
        for (int c = 0; c < copies; ++c)
            s += lds_hist[c * PER_COPY + i];
        if (s)
            atomicAdd(&hist[i], (unsigned long long)s);
    }
}

// Exclusive prefix over tiles of per-tile digit counts (256 digits, one
// thread per digit), in three steps over blocks of kTilePrefixBlock tiles:
// block sums, an exclusive scan of the block sums per digit, and the
// in-place rewrite of each block's counts into prefixes.
// Tiles whose counts one thread has in flight at once in the prefix kernels.
constexpr uint32_t kTilePrefixBatch = 16;
static_assert(kTilePrefixBlock % kTilePrefixBatch == 0, "whole batches per block");

template <typename ST>
__global__ __launch_bounds__(256) void tile_block_sum_kernel(const ST* __restrict__ counts, uint32_t tiles,
                                                            uint64_t* __restrict__ block_sums)
{
    const uint32_t t0 = blockIdx.x * kTilePrefixBlock;
    const uint32_t t1 = t0 + kTilePrefixBlock < tiles ? t0 + kTilePrefixBlock : tiles;
    uint64_t s = 0;
    for (uint32_t tb = t0; tb < t1; tb += kTilePrefixBatch) {
        ST c[kTilePrefixBatch];
#pragma unroll
        for (uint32_t j = 0; j < kTilePrefixBatch; ++j)
            c[j] = counts[(size_t)(tb + j < t1 ? tb + j : t1 - 1) * 256 + threadIdx.x];  // no branch
#pragma unroll
        for (uint32_t j = 0; j < kTilePrefixBatch; ++j)
            s += tb + j < t1 ? (uint64_t)c[j] : 0;
    }
    block_sums[(size_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// One workgroup per digit: exclusive scan of block_sums[.][digit] in place.
template <int THREADS>
__global__ __launch_bounds__(THREADS) void tile_block_scan_kernel(uint64_t* __restrict__ block_sums, uint32_t blocks)
{
    static_assert(THREADS == 256, "one thread per digit");
    __shared__ uint64_t part[256];
    const uint32_t d = blockIdx.x;
    const uint32_t per = (blocks + 255) / 256;
    const uint32_t b0 = threadIdx.x * per;
    uint64_t s = 0;
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < blocks)
            s += block_sums[(size_t)(b0 + j) * 256 + d];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 256; o <<= 1) {
        const uint64_t y = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - s;
    for (uint32_t j = 0; j < per; ++j)
        if (b0 + j < blocks) {
            uint64_t* p = &block_sums[(size_t)(b0 + j) * 256 + d];
            const uint64_t c = *p;
            *p = run;
            run += c;
        }
}

template <typename ST>
__global__ __launch_bounds__(256) void tile_prefix_kernel(ST* __restrict__ counts, uint32_t tiles,
                                                         const uint64_t* __restrict__ block_sums)
{
    const uint32_t t0 = blockIdx.x * kTilePrefixBlock;
    const uint32_t t1 = t0 + kTilePrefixBlock < tiles ? t0 + kTilePrefixBlock : tiles;
    uint64_t run = block_sums[(size_t)blockIdx.x * 256 + threadIdx.x];
    for (uint32_t tb = t0; tb < t1; tb += kTilePrefixBatch) {
        ST c[kTilePrefixBatch];
#pragma unroll
        for (uint32_t j = 0; j < kTilePrefixBatch; ++j)
            c[j] = counts[(size_t)(tb + j < t1 ? tb + j : t1 - 1) * 256 + threadIdx.x];  // no branch
#pragma unroll
        for (uint32_t j = 0; j < kTilePrefixBatch; ++j) {
            if (tb + j < t1) {
                counts[(size_t)(tb + j) * 256 + threadIdx.x] = (ST)run;
                run += (uint64_t)c[j];
            }
        }
    }
}

// ------------------------------------------------------------------------
// Digit bases: exclusive scan of one histogram row per workgroup; with
// `live` (one word, zeroed before), bit p set when pass p's digit takes more
// than one value (a row whose whole count sits in one digit leaves the order
// unchanged: its pass can go)
// ------------------------------------------------------------------------
template <int THREADS>
__global__ __launch_bounds__(THREADS) void radix_scan_kernel(const uint64_t* __restrict__ hist,
                                                             uint64_t* __restrict__ bases, int bins,
                                                             uint32_t* __restrict__ live, uint32_t* done,
                                                             unsigned long long* tickets)
{
    __shared__ uint64_t part[THREADS];
    __shared__ uint32_t one_digit;
    if (threadIdx.x == 0)
        one_digit = 0;
    const uint64_t* row = hist + (size_t)blockIdx.x * bins;
    uint64_t* out = bases + (size_t)blockIdx.x * bins;
    const int per = (bins + THREADS - 1) / THREADS;
    const int b0 = threadIdx.x * per;
    uint64_t s = 0;
    for (int j = 0; j < per; ++j)
        if (b0 + j < bins)
            s += row[b0 + j];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over THREADS partial sums.
    for (int o = 1; o < THREADS; o <<= 1) {
        uint64_t y = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += y;
        __syncthreads();
    }
    uint64_t run = part[threadIdx.x] - s;
    const uint64_t total = part[THREADS - 1];
    for (int j = 0; j < per; ++j)
        if (b0 + j < bins) {
            const uint64_t c = row[b0 + j];
            out[b0 + j] = run;
            run += c;
            if (c == total)
                one_digit = 1;  // every key has this digit
        }
    __syncthreads();
    if (!live || threadIdx.x != 0)
        return;
    if (!one_digit)
        atomicOr(live, 1u << blockIdx.x);
    // The last workgroup to finish writes every pass's route code into the
    // upper half of its ticket counter, so that a pass learns its route from
    // the ticket it takes anyway.
    __threadfence();
    if (atomicAdd(done, 1u) != gridDim.x - 1)
        return;
    __threadfence();
    const uint32_t mask = __hip_atomic_load(live, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t m = (uint32_t)__builtin_popcount(mask);
    for (uint32_t q = 0; q < gridDim.x; ++q) {
        const uint32_t j = (uint32_t)__builtin_popcount(mask & ((1u << q) - 1u));
        tickets[q] = (unsigned long long)route_code((mask >> q) & 1u, j, m) << 32;
    }
}

// ------------------------------------------------------------------------
// Look-back status words: 2 flag bits above the count.
// ------------------------------------------------------------------------
template <typename ST>
struct Status;
template <>
struct Status<uint32_t> {
    static constexpr int kShift = 30;  // counts < 2^30: used only when n < 2^30
    static constexpr uint32_t kMask = (1u << 30) - 1;
};
template <>
struct Status<uint64_t> {
    static constexpr int kShift = 62;
    static constexpr uint64_t kMask = (1ull << 62) - 1;
};
constexpr uint32_t kFlagAggregate = 1;  // count of this tile only
constexpr uint32_t kFlagInclusive = 2;  // count of this tile and every tile before it

// Number of predecessor look-back words read at once.  Each agent-scope read
// crosses to memory (the XCDs' L2s are not coherent with each other), so the
// walk reads several predecessors per round trip.
constexpr int kLookBackWindow = 4;

// Sum of digit b's counts over tiles [0, tile): walk back from tile - 1,
// reading kLookBackWindow words per round trip, adding aggregates until an
// inclusive word ends the walk.  An unpublished word is polled (bounded by
// spin_limit; running out sets *error_word, and *host_error when given, and
// returns what was summed).
// Tile 0 always publishes an inclusive word, so the walk never passes it;
// window slots before tile 0 re-read tile 0's word (in bounds, never used
// past it).
template <typename ST, int BINS>
__device__ __forceinline__ uint64_t look_back(const ST* status, uint32_t tile, int b, uint32_t spin_limit,
                                              uint32_t* error_word, uint32_t* host_error)
{
    constexpr int W = kLookBackWindow;
    uint64_t excl = 0;
    int32_t t = (int32_t)tile - 1;
    uint32_t spins = 0;
    for (;;) {
        ST s[W];
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const int32_t tt = t - w > 0 ? t - w : 0;
            s[w] = load_agent(&status[(size_t)(uint32_t)tt * BINS + b]);
        }
        int stop = W;  // window slot to wait on; W: none
        bool done = false;
#pragma unroll
        for (int w = W - 1; w >= 0; --w) {
            // scanning from the far end keeps the nearest unpublished slot
            const uint32_t flag = (uint32_t)(s[w] >> Status<ST>::kShift);
            if (flag == 0)
                stop = w;
        }
#pragma unroll
        for (int w = 0; w < W; ++w) {
            if (!done && w < stop) {
                excl += (uint64_t)(s[w] & Status<ST>::kMask);
                done = (uint32_t)(s[w] >> Status<ST>::kShift) == kFlagInclusive;
            }
        }
        if (done)
            return excl;
        if (stop == W) {
            t -= W;
            continue;
        }
        t -= stop;
        ST x;
        while (((x = load_agent(&status[(size_t)(uint32_t)t * BINS + b])) >> Status<ST>::kShift) == 0) {
            if (++spins > spin_limit) {
                atomicOr(error_word, kDeviceErrTimeout);
                report_host_error(host_error, kDeviceErrTimeout);
                return excl;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        excl += (uint64_t)(x & Status<ST>::kMask);
        if ((uint32_t)(x >> Status<ST>::kShift) == kFlagInclusive)
            return excl;
        --t;
    }
}

// ------------------------------------------------------------------------
// One single-sweep LSD pass
// ------------------------------------------------------------------------
// Tile layout: a workgroup of THREADS threads owns TILE = THREADS*ITEMS
// consecutive keys.  Wave w owns the sub-range [w*64*ITEMS, (w+1)*64*ITEMS)
// and its item i is lane-striped: key w*64*ITEMS + i*64 + lane.  Processing
// items in order i = 0, 1, ... and lanes in order inside an item therefore
// visits the tile's keys in input order, which is what makes the rank stable.

// LDS of one pass workgroup.  The per-wave digit counters and the output
// staging area are never live at the same time, so they share storage.
template <int KB, int VB, int BITS, int THREADS, int ITEMS>
struct PassLds {
    static constexpr int BINS = 1 << BITS;
    static constexpr int WAVES = THREADS / kWave;
    static constexpr int TILE = THREADS * ITEMS;
    // counters [WAVES][BINS] uint32, then (digits up to 11 bits) lane
    // buckets [WAVES][BINS] uint64
    static constexpr bool kBuckets = BITS <= 11;
    static constexpr size_t BUCKET_OFFSET = ((size_t)WAVES * BINS * 4 + 15) & ~(size_t)15;
    static constexpr size_t HIST_BYTES = BUCKET_OFFSET + (kBuckets ? (size_t)WAVES * BINS * 8 : 0);
    static constexpr size_t STAGE_BYTES = (size_t)TILE * KB + (size_t)(VB ? TILE * VB : 0);
    static constexpr size_t UNION_BYTES = HIST_BYTES > STAGE_BYTES ? HIST_BYTES : STAGE_BYTES;
    __attribute__((aligned(16))) unsigned char uni[UNION_BYTES];
    int64_t gofs[BINS];  // output slot of tile position 0, per digit (32-bit values while n < 2^30)
    uint32_t wtot[WAVES];
    unsigned long long ticket;  // the workgroup's ticket (route code and tile), shared from the lane that took it
};

// Everything a workgroup does for one tile after it has its tile number.
// FULL: the tile holds TILE keys (every tile but possibly the last), so no
// per-item validity is tracked.
// The buffers and per-pass flags one pass works with (the kernel's own
// arguments, or what the route picks for it).
struct PassIo {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;
    void* vals_out;
    uint32_t flags;  // RADIX_FLAG_*
};

template <bool FULL, int KB, int VB, int BITS, int THREADS, int ITEMS, typename ST>
__device__ __forceinline__ void pass_tile(const RadixPassArgs& a, const PassIo& io,
                                          const OrderMap<typename KeyWord<KB>::U>& om,
                                          PassLds<KB, VB, BITS, THREADS, ITEMS>& L, uint32_t tile, int64_t tile_start,
                                          uint32_t nvalid)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using Lds = PassLds<KB, VB, BITS, THREADS, ITEMS>;
    constexpr int BINS = 1 << BITS;
    constexpr int WAVES = THREADS / kWave;
    constexpr int TILE = THREADS * ITEMS;
    constexpr int WAVE_KEYS = kWave * ITEMS;
    constexpr int BPT = (BINS + THREADS - 1) / THREADS;  // bins per thread
    // With 32-bit look-back words n < 2^30, so output slots fit in 32 bits.
    constexpr bool kOff32 = sizeof(ST) == 4;

    uint32_t* s_whist = reinterpret_cast<uint32_t*>(L.uni);  // [WAVES][BINS]
    U* s_keys = reinterpret_cast<U*>(L.uni);
    V* s_vals = reinterpret_cast<V*>(L.uni + (size_t)TILE * KB);
    ST* status = reinterpret_cast<ST*>(a.status);

    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    // Offsets inside the tile are 32-bit; only the tile base is 64-bit.
    const uint32_t off0 = (uint32_t)(w * WAVE_KEYS + lane);
    const U* __restrict__ tile_keys = reinterpret_cast<const U*>(io.keys_in) + tile_start;
    // item i of this thread is valid iff i * 64 < rem: one register for all
    // items instead of one offset per item
    const int32_t rem = FULL ? 0 : (int32_t)materialize(nvalid - off0);
    auto item_valid = [&](int i) { return FULL || (int32_t)(i * kWave) < rem; };

    // ---- load ----------------------------------------------------------
    // Past the end of the last tile the load is clamped to the last key (in
    // bounds, no branch); such items are excluded from the rank below.
    U k[ITEMS];
    V v[VB ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t off = off0 + (uint32_t)(i * kWave);
        k[i] = load_off32(tile_keys, FULL ? off : min(off, nvalid - 1));
    }
    if constexpr (VB != 0) {
        const V* __restrict__ tile_vals = reinterpret_cast<const V*>(io.vals_in) + tile_start;
        const bool iota = (io.flags & RADIX_FLAG_IOTA) != 0;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t off = off0 + (uint32_t)(i * kWave);
            if (iota)
                v[i] = (V)(tile_start + off);
            else
                v[i] = load_off32(tile_vals, FULL ? off : min(off, nvalid - 1));
        }
    }

    // Zero the wave counters and buckets while the loads are in flight (the
    // previous tile's write-out finished reading this storage at the barrier
    // that ended it).
    for (int i = threadIdx.x; i < WAVES * BINS; i += THREADS)
        s_whist[i] = 0;
    if constexpr (Lds::kBuckets) {
        uint64_t* s_bkt = reinterpret_cast<uint64_t*>(L.uni + Lds::BUCKET_OFFSET);
        for (int i = threadIdx.x; i < WAVES * BINS; i += THREADS)
            s_bkt[i] = 0;
    }
    __syncthreads();

    // ---- stable rank inside each wave ------------------------------------
    // Items are visited in order.  For item i every valid lane ORs its lane
    // bit into the wave's 64-bit bucket of its digit, then reads the bucket
    // back: the bits are exactly the lanes of this item holding the same
    // digit (OR is order-independent, and one wave's LDS instructions run in
    // program order).  Each lane also reads the wave's running count for its
    // digit; the lowest lane of the group then clears the bucket (a no-op for
    // lane 0's group, which never sets it) and adds the group size to the
    // count.
    // rk holds each key's rank among the wave's equal digits, 16 bits per
    // key, two keys per word (the digit is recomputed from the key later):
    // fewer live registers, so more workgroups fit on a CU.
    uint32_t* wh = s_whist + w * BINS;
    constexpr int PAIRS = (ITEMS + 1) / 2;
    uint32_t rk[PAIRS];
    auto put_rank = [&](int i, uint32_t r) {
        // materialized now: a deferred pack would keep its operands alive
        rk[i >> 1] = (i & 1) ? materialize(rk[i >> 1] | (r << 16)) : materialize(r);
    };
    if constexpr (Lds::kBuckets) {
        uint64_t* bkt = reinterpret_cast<uint64_t*>(L.uni + Lds::BUCKET_OFFSET) + w * BINS;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t d = (uint32_t)((om.to_order(k[i]) >> a.shift) & (U)(BINS - 1));
            const bool valid = item_valid(i);
            // The lanes holding lane 0's digit know their peers from one
            // ballot and leave the bucket alone: with skewed, presorted or
            // sparse keys they are most of the wave, and their bucket atomics
            // would be executed one lane at a time.  The other lanes set
            // their bit in the 32-bit half of their digit's bucket.
            const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
            const uint64_t same = ballot(d == d0);
            const uint64_t vmask = FULL ? ~0ull : ballot(valid);
            if (same != ~0ull && d != d0 && (FULL || valid))
                atomicOr(reinterpret_cast<uint32_t*>(&bkt[d]) + (lane >> 5), 1u << (lane & 31));
            const uint64_t peers = d == d0 ? (same & vmask) : bkt[d];
            const uint32_t old = wh[d];
            const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(peers >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((uint32_t)peers, 0u));
            if ((FULL || valid) && below == 0) {
                bkt[d] = 0;
                wh[d] = old + (uint32_t)__popcll(peers);
            }
            put_rank(i, old + below);
        }
    } else {
        // Wide digits (the buckets would not fit in LDS): the same peer mask
        // from one ballot per digit bit; a lane keeps the lanes whose bit
        // equals its own (peers &= ~(ballot ^ sel), sel = all ones when set).
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            uint32_t d = (uint32_t)((om.to_order(k[i]) >> a.shift) & (U)(BINS - 1));
            // Item i's ballots start after item i-1's result: otherwise the
            // compiler hoists every item's 64-bit ballots and spills them.
            if (i > 0)
                d = after(d, rk[(i - 1) >> 1]);
            const bool valid = item_valid(i);
            const uint64_t vmask = FULL ? ~0ull : ballot(valid);
            uint32_t plo = (uint32_t)vmask, phi = (uint32_t)(vmask >> 32);
#pragma unroll
            for (int b = 0; b < BITS; ++b) {
                const uint32_t sel = bit_mask_of(d, b);
                const uint64_t m = ballot(sel != 0);
                plo = keep_equal_bits(plo, (uint32_t)m, sel);
                phi = keep_equal_bits(phi, (uint32_t)(m >> 32), sel);
            }
            const uint32_t below = __builtin_amdgcn_mbcnt_hi(phi, __builtin_amdgcn_mbcnt_lo(plo, 0u));
            const uint32_t old = wh[d];
            if ((FULL || valid) && below == 0)
                wh[d] = old + (uint32_t)(__builtin_popcount(plo) + __builtin_popcount(phi));
            put_rank(i, old + below);
        }
    }
    __syncthreads();

    // ---- tile counts, publication, in-tile scan ----------------------------
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
    const bool prefixed = (io.flags & RADIX_FLAG_PREFIX) != 0;
    const bool publish = !prefixed && !((io.flags & RADIX_FLAG_WITHHOLD_T0) && tile == 0);
    if (publish) {
        const ST flag = (ST)(tile == 0 ? kFlagInclusive : kFlagAggregate) << Status<ST>::kShift;
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = threadIdx.x * BPT + j;
            if (b < BINS)
                store_agent(&status[(size_t)tile * BINS + b], (ST)(flag | (ST)cnt[j]));
        }
    }
    uint32_t tile_total;
    const uint32_t first = block_exclusive_scan<THREADS>(tsum, L.wtot, &tile_total);
    (void)tile_total;

    // Turn each wave's digit counts into the wave's first local position.
    uint32_t start[BPT];
    {
        uint32_t run = first;
#pragma unroll
        for (int j = 0; j < BPT; ++j) {
            const int b = threadIdx.x * BPT + j;
            start[j] = run;
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
    }

    __syncthreads();  // every wave's first local positions are in LDS

    // ---- local positions, then stage the tile in digit order ----------------
    // Done before the look-back so that predecessors get more time to publish.
    // Positions in the tile are below 2^16 and replace the ranks in place,
    // two per word; 0xffff marks an item past the end of the last tile.
#pragma unroll
    for (int j = 0; j < PAIRS; ++j) {
        uint32_t packed = 0;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int i = 2 * j + h;
            if (i < ITEMS) {
                const uint32_t d = (uint32_t)((om.to_order(k[i]) >> a.shift) & (U)(BINS - 1));
                const uint32_t pos =
                    item_valid(i) ? s_whist[w * BINS + d] + ((rk[j] >> (16 * h)) & 0xffffu) : 0xffffu;
                packed |= pos << (16 * h);
            }
        }
        rk[j] = materialize(packed);
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t pos = (rk[i >> 1] >> (16 * (i & 1))) & 0xffffu;
        if (FULL || pos != 0xffffu) {
            s_keys[pos] = k[i];
            if constexpr (VB != 0)
                s_vals[pos] = v[i];
        }
    }

    // ---- decoupled look-back per digit -------------------------------------
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = threadIdx.x * BPT + j;
        if (b >= BINS)
            continue;
        uint64_t excl = 0;
        if (prefixed) {
            excl = (uint64_t)status[(size_t)tile * BINS + b];  // written before this kernel
        } else if (tile > 0) {
            excl = look_back<ST, BINS>(status, tile, b, a.spin_limit, a.error_word, a.host_error);
            store_agent(&status[(size_t)tile * BINS + b],
                        (ST)(((ST)kFlagInclusive << Status<ST>::kShift) | (ST)(excl + cnt[j])));
        }
        const int64_t g = (int64_t)(a.bases[b] + excl) - (int64_t)start[j];
        if constexpr (kOff32)
            reinterpret_cast<int32_t*>(L.gofs)[b] = (int32_t)g;
        else
            L.gofs[b] = g;
    }
    __syncthreads();  // staged keys and per-digit output slots are in LDS

    // ---- coalesced write-out: consecutive threads, consecutive positions ----
    const bool write_keys = !(io.flags & RADIX_FLAG_SKIP_KEYS);
    U* __restrict__ keys_out = reinterpret_cast<U*>(io.keys_out);
    V* __restrict__ vals_out = reinterpret_cast<V*>(io.vals_out);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = (uint32_t)(i * THREADS) + threadIdx.x;
        if (FULL || p < nvalid) {
            const U key = s_keys[p];
            const uint32_t d = (uint32_t)((om.to_order(key) >> a.shift) & (U)(BINS - 1));
            // dst is in [0, n) whenever the histogram matches the keys; the
            // bounds check keeps a broken invariant from becoming a wild store.
            if constexpr (kOff32) {
                const uint32_t dst = (uint32_t)(reinterpret_cast<const int32_t*>(L.gofs)[d] + (int32_t)p);
                if (dst < (uint32_t)a.n) {
                    if (write_keys)
                        keys_out[dst] = key;
                    if constexpr (VB != 0)
                        vals_out[dst] = s_vals[p];
                }
            } else {
                const int64_t dst = L.gofs[d] + p;
                if ((uint64_t)dst < (uint64_t)a.n) {
                    if (write_keys)
                        keys_out[dst] = key;
                    if constexpr (VB != 0)
                        vals_out[dst] = s_vals[p];
                }
            }
        }
    }
}

// A routed pass (see RadixRoute) picks its buffers from its route code: live
// pass j of m live passes.
__device__ __forceinline__ void route_pass(const RadixRoute& r, uint32_t j, uint32_t m, PassIo& io)
{
    if (r.flags & ROUTE_ARGSORT) {
        const bool to_out = ((m - 1 - j) & 1) == 0;
        io.keys_in = j == 0 ? r.keys_in : (((j - 1) & 1) ? r.keys_tmp2 : r.keys_tmp);
        io.keys_out = (j & 1) ? r.keys_tmp2 : r.keys_tmp;
        io.vals_out = to_out ? r.vals_out : r.vals_tmp;
        io.vals_in = j == 0 ? nullptr : (to_out ? r.vals_tmp : r.vals_out);
        io.flags |= (j == 0 ? RADIX_FLAG_IOTA : 0u) | (j == m - 1 ? RADIX_FLAG_SKIP_KEYS : 0u);
    } else {
        // whether live pass jj writes the output (else the temporary buffer)
        const bool odd_copy = (r.flags & ROUTE_COPY_IF_ODD) && (m & 1);
        const bool out_now = odd_copy ? (j & 1) != 0 : ((m - 1 - j) & 1) == 0;
        const bool out_before = j > 0 && (odd_copy ? ((j - 1) & 1) != 0 : ((m - j) & 1) == 0);
        io.keys_out = out_now ? r.keys_out : r.keys_tmp;
        io.keys_in = j == 0 ? r.keys_in : (out_before ? r.keys_out : r.keys_tmp);
        io.vals_out = out_now ? r.vals_out : r.vals_tmp;
        io.vals_in = j == 0 ? r.vals_in : (out_before ? r.vals_out : r.vals_tmp);
    }
}

// One workgroup per tile.  The tile number is a ticket taken from an atomic
// counter, not blockIdx: tickets are handed out in the order workgroups start
// running, so a tile's look-back only ever waits on tiles whose workgroups are
// already resident, and every wait ends.
template <int KB, int VB, int BITS, int THREADS, int ITEMS, typename ST>
__global__ __launch_bounds__(THREADS) void radix_pass_kernel(RadixPassArgs a, OrderMap<typename KeyWord<KB>::U> om)
{
    using Lds = PassLds<KB, VB, BITS, THREADS, ITEMS>;
    constexpr int TILE = THREADS * ITEMS;
    static_assert(THREADS * ITEMS < 65535, "tile positions are 16 bits");
    static_assert((1 << BITS) <= 4096, "digit field is 12 bits");
    __shared__ Lds L;

    // The ticket's lower half is the tile; its upper half is the pass's route
    // code, which the scan kernel wrote into the counter (0: not routed).
    if (threadIdx.x == 0)
        L.ticket = atomicAdd(a.ticket, 1ull);
    // The route's buffers are kernel arguments: have them in scalar registers
    // while the ticket is in flight, not requested once it has arrived (the
    // tile's loads wait on the choice).
    in_sgprs(a.route.flags);
    in_sgprs(a.route.keys_in);
    in_sgprs(a.route.keys_out);
    in_sgprs(a.route.keys_tmp);
    if constexpr (VB != 0) {
        in_sgprs(a.route.keys_tmp2);
        in_sgprs(a.route.vals_in);
        in_sgprs(a.route.vals_out);
        in_sgprs(a.route.vals_tmp);
    }
    __syncthreads();
    const unsigned long long t = L.ticket;
    const uint32_t code = __builtin_amdgcn_readfirstlane((uint32_t)(t >> 32));
    const uint32_t tile = __builtin_amdgcn_readfirstlane((uint32_t)t);
    PassIo io{a.keys_in, a.keys_out, a.vals_in, a.vals_out, a.flags};
    if (code & kRouteOn) {
        if (!(code & kRouteLive))
            return;  // uniform: this pass's digit is the same for every key
        route_pass(a.route, route_j(code), route_m(code), io);
    }
    if (tile >= a.tiles)
        return;  // uniform across the workgroup
    const int64_t tile_start = (int64_t)tile * TILE;
    const int64_t left = a.n - tile_start;
    if (left >= TILE)
        pass_tile<true, KB, VB, BITS, THREADS, ITEMS, ST>(a, io, om, L, tile, tile_start, (uint32_t)TILE);
    else
        pass_tile<false, KB, VB, BITS, THREADS, ITEMS, ST>(a, io, om, L, tile, tile_start, (uint32_t)left);
}

// One pass over the tiles of every large segment of a batched sort.  Tiles
// are numbered globally, each segment's tiles consecutively, and handed out by
// the ticket in that order.  A tile sees its segment as a whole array: its
// keys, its digit bases and its look-back words start at the segment's first
// key and first tile, so the chained scan of a segment starts at its own
// first tile.  Exactly *tile_count workgroups take a ticket.
template <int KB, int VB, int BITS, int THREADS, int ITEMS>
__global__ __launch_bounds__(THREADS) void seg_radix_pass_kernel(SegPassArgs sa,
                                                                 OrderMap<typename KeyWord<KB>::U> om)
{
    using ST = uint32_t;  // segments hold fewer than 2^30 keys
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using Lds = PassLds<KB, VB, BITS, THREADS, ITEMS>;
    constexpr int TILE = THREADS * ITEMS;
    constexpr int BINS = 1 << BITS;
    __shared__ Lds L;

    if (blockIdx.x >= *sa.tile_count)
        return;  // uniform across the workgroup
    if (threadIdx.x == 0)
        L.ticket = atomicAdd(sa.base.tile_counter, 1u);
    __syncthreads();
    // The ticket is the same in every lane; saying so (and the same for the
    // segment's fields) keeps the segment's description and pointers in
    // scalar registers.
    const uint32_t t = __builtin_amdgcn_readfirstlane((uint32_t)L.ticket);
    const uint32_t slot = __builtin_amdgcn_readfirstlane(sa.tile_slot[t]);
    SegLarge g = sa.large[slot];
    g.begin = (int64_t)(((uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)g.begin >> 32)) << 32) |
                        (uint64_t)__builtin_amdgcn_readfirstlane((uint32_t)g.begin));
    g.len = __builtin_amdgcn_readfirstlane(g.len);
    g.first_tile = __builtin_amdgcn_readfirstlane(g.first_tile);
    RadixPassArgs a = sa.base;
    PassIo io{reinterpret_cast<const U*>(sa.base.keys_in) + g.begin, reinterpret_cast<U*>(sa.base.keys_out) + g.begin,
              nullptr, nullptr, sa.base.flags};
    if constexpr (VB != 0) {
        io.vals_in = reinterpret_cast<const V*>(sa.base.vals_in) + g.begin;
        io.vals_out = reinterpret_cast<V*>(sa.base.vals_out) + g.begin;
    }
    a.n = g.len;
    a.bases = sa.base.bases + (size_t)slot * sa.slot_stride;
    a.status = reinterpret_cast<ST*>(sa.base.status) + (size_t)g.first_tile * BINS;
    const uint32_t lt = t - g.first_tile;
    const int64_t tile_start = (int64_t)lt * TILE;
    const int64_t left = (int64_t)g.len - tile_start;
    if (left >= TILE)
        pass_tile<true, KB, VB, BITS, THREADS, ITEMS, ST>(a, io, om, L, lt, tile_start, (uint32_t)TILE);
    else
        pass_tile<false, KB, VB, BITS, THREADS, ITEMS, ST>(a, io, om, L, lt, tile_start, (uint32_t)left);
}

template <int KB, int VB, int BITS, int THREADS, int ITEMS, typename ST>
hipError_t launch_radix_pass_t(const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL((radix_pass_kernel<KB, VB, BITS, THREADS, ITEMS, ST>), dim3(tiles), dim3(THREADS), 0, s, a,
                       om);
    return hipGetLastError();
}

template <int KB, int VB, int BITS, int THREADS, int ITEMS>
hipError_t launch_seg_radix_pass_t(const KeyDesc& kd, const SegPassArgs& a, uint32_t grid, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    if (grid == 0)
        return hipSuccess;
    hipLaunchKernelGGL((seg_radix_pass_kernel<KB, VB, BITS, THREADS, ITEMS>), dim3(grid), dim3(THREADS), 0, s, a, om);
    return hipGetLastError();
}

}  // namespace evosort
