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
    const int64_t stride = (int64_t)gridDim.x * THREADS;
    const int64_t gtid = (int64_t)blockIdx.x * THREADS + threadIdx.x;
    int64_t done = 0;
    if ((reinterpret_cast<uintptr_t>(keys) & 15) == 0) {
        const int64_t nvec = n / VEC;
        const uint4* kv = reinterpret_cast<const uint4*>(keys);
        for (int64_t v = gtid; v < nvec; v += stride) {
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

// ------------------------------------------------------------------------
// Digit bases: exclusive scan of one histogram row per workgroup
// ------------------------------------------------------------------------
template <int THREADS>
__global__ __launch_bounds__(THREADS) void radix_scan_kernel(const uint64_t* __restrict__ hist,
                                                             uint64_t* __restrict__ bases, int bins)
{
    __shared__ uint64_t part[THREADS];
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
    for (int j = 0; j < per; ++j)
        if (b0 + j < bins) {
            out[b0 + j] = run;
            run += row[b0 + j];
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

// ------------------------------------------------------------------------
// One single-sweep LSD pass
// ------------------------------------------------------------------------
// Tile layout: a workgroup of THREADS threads owns TILE = THREADS*ITEMS
// consecutive keys.  Wave w owns the sub-range [w*64*ITEMS, (w+1)*64*ITEMS)
// and its item i is lane-striped: key w*64*ITEMS + i*64 + lane.  Processing
// items in order i = 0, 1, ... and lanes in order inside an item therefore
// visits the tile's keys in input order, which is what makes the rank stable.
template <int KB, int VB, int BITS, int THREADS, int ITEMS, typename ST>
__global__ __launch_bounds__(THREADS) void radix_pass_kernel(RadixPassArgs a, OrderMap<typename KeyWord<KB>::U> om)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    constexpr int BINS = 1 << BITS;
    constexpr int WAVES = THREADS / kWave;
    constexpr int TILE = THREADS * ITEMS;
    constexpr int WAVE_KEYS = kWave * ITEMS;
    constexpr int BPT = (BINS + THREADS - 1) / THREADS;  // bins per thread
    constexpr size_t HIST_BYTES = (size_t)WAVES * BINS * 4;
    constexpr size_t STAGE_BYTES = (size_t)TILE * KB + (size_t)(VB ? TILE * VB : 0);
    constexpr size_t UNION_BYTES = HIST_BYTES > STAGE_BYTES ? HIST_BYTES : STAGE_BYTES;
    static_assert(WAVE_KEYS < 65536, "rank field is 16 bits");
    static_assert(BINS <= 4096, "digit field is 12 bits");

    // The per-wave digit counters and the output staging area are never live
    // at the same time, so they share LDS.
    __shared__ __attribute__((aligned(16))) unsigned char s_union[UNION_BYTES];
    __shared__ int64_t s_gofs[BINS];  // output slot of tile position 0 for each digit
    __shared__ uint32_t s_wtot[WAVES];
    __shared__ uint32_t s_tile;

    uint32_t* s_whist = reinterpret_cast<uint32_t*>(s_union);  // [WAVES][BINS]
    U* s_keys = reinterpret_cast<U*>(s_union);
    V* s_vals = reinterpret_cast<V*>(s_union + (size_t)TILE * KB);

    const U* __restrict__ keys_in = reinterpret_cast<const U*>(a.keys_in);
    U* __restrict__ keys_out = reinterpret_cast<U*>(a.keys_out);
    ST* status = reinterpret_cast<ST*>(a.status);

    // Tiles are handed out in launch order, so a tile only ever waits on tiles
    // whose workgroups are already running.
    if (threadIdx.x == 0)
        s_tile = atomicAdd(a.tile_counter, 1u);
    for (int i = threadIdx.x; i < WAVES * BINS; i += THREADS)
        s_whist[i] = 0;
    __syncthreads();

    const uint32_t tile = s_tile;
    if (tile >= a.tiles)
        return;  // uniform across the workgroup: cannot happen with a zeroed counter
    const int64_t tile_start = (int64_t)tile * TILE;
    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const int64_t my0 = tile_start + (int64_t)w * WAVE_KEYS + lane;
    const bool full = tile_start + TILE <= a.n;

    // ---- load ----------------------------------------------------------
    U k[ITEMS];
    V v[VB ? ITEMS : 1];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int64_t idx = my0 + (int64_t)i * kWave;
        k[i] = (full || idx < a.n) ? keys_in[idx] : (U)0;
    }
    if constexpr (VB != 0) {
        const V* __restrict__ vals_in = reinterpret_cast<const V*>(a.vals_in);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const int64_t idx = my0 + (int64_t)i * kWave;
            if (a.flags & RADIX_FLAG_IOTA)
                v[i] = (V)idx;
            else
                v[i] = (full || idx < a.n) ? vals_in[idx] : (V)0;
        }
    }

    // ---- stable rank inside each wave ------------------------------------
    // For item i, the lanes holding the same digit are found with one ballot
    // per digit bit; the lowest such lane bumps the wave's counter for that
    // digit after all of them read it.  rk = digit << 16 | rank within wave.
    uint32_t rk[ITEMS];
    uint32_t* wh = s_whist + w * BINS;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = full || (my0 + (int64_t)i * kWave < a.n);
        const uint32_t d = (uint32_t)((om.to_order(k[i]) >> a.shift) & (U)(BINS - 1));
        uint64_t peers = ballot(valid);
#pragma unroll
        for (int b = 0; b < BITS; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t below = lanes_below(peers);
        uint32_t old = 0;
        if (valid) {
            old = wh[d];
            if (below == 0)
                wh[d] = old + (uint32_t)__popcll(peers);
        }
        rk[i] = (d << 16) | (old + below);
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
    const bool publish = !((a.flags & RADIX_FLAG_WITHHOLD_T0) && tile == 0);
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
    const uint32_t first = block_exclusive_scan<THREADS>(tsum, s_wtot, &tile_total);
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

    // ---- decoupled look-back per digit -------------------------------------
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
        const int b = threadIdx.x * BPT + j;
        if (b >= BINS)
            continue;
        uint64_t excl = 0;
        if (tile > 0) {
            int64_t t = (int64_t)tile - 1;
            uint32_t spins = 0;
            while (true) {
                const ST s = load_agent(&status[(size_t)t * BINS + b]);
                const uint32_t flag = (uint32_t)(s >> Status<ST>::kShift);
                if (flag == 0) {
                    if (++spins > a.spin_limit) {
                        atomicOr(a.error_word, 1u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                excl += (uint64_t)(s & Status<ST>::kMask);
                if (flag == kFlagInclusive || t == 0)
                    break;
                --t;
            }
            store_agent(&status[(size_t)tile * BINS + b],
                        (ST)(((ST)kFlagInclusive << Status<ST>::kShift) | (ST)(excl + cnt[j])));
        }
        s_gofs[b] = (int64_t)(a.bases[b] + excl) - (int64_t)start[j];
    }
    __syncthreads();

    // ---- local positions, then stage the tile in digit order ----------------
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const bool valid = full || (my0 + (int64_t)i * kWave < a.n);
        rk[i] = valid ? s_whist[w * BINS + (rk[i] >> 16)] + (rk[i] & 0xffffu) : 0xffffffffu;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        if (rk[i] != 0xffffffffu) {
            s_keys[rk[i]] = k[i];
            if constexpr (VB != 0)
                s_vals[rk[i]] = v[i];
        }
    }
    __syncthreads();

    // ---- coalesced write-out: consecutive threads, consecutive positions ----
    const int nvalid = full ? TILE : (int)(a.n - tile_start);
    const bool write_keys = !(a.flags & RADIX_FLAG_SKIP_KEYS);
    V* __restrict__ vals_out = reinterpret_cast<V*>(a.vals_out);
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const int p = i * THREADS + threadIdx.x;
        if (p < nvalid) {
            const U key = s_keys[p];
            const uint32_t d = (uint32_t)((om.to_order(key) >> a.shift) & (U)(BINS - 1));
            const int64_t dst = s_gofs[d] + p;
            // dst is in [0, n) whenever the histogram matches the keys; the
            // check keeps a broken invariant from becoming a wild store.
            if ((uint64_t)dst < (uint64_t)a.n) {
                if (write_keys)
                    keys_out[dst] = key;
                if constexpr (VB != 0)
                    vals_out[dst] = s_vals[p];
            }
        }
    }
}

template <int KB, int VB, int BITS, int THREADS, int ITEMS, typename ST>
hipError_t launch_radix_pass_t(const KeyDesc& kd, const RadixPassArgs& a, uint32_t tiles, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg};
    hipLaunchKernelGGL((radix_pass_kernel<KB, VB, BITS, THREADS, ITEMS, ST>), dim3(tiles), dim3(THREADS), 0, s, a,
                       om);
    return hipGetLastError();
}

}  // namespace evosort
