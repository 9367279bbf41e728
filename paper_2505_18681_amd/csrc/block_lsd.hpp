// One-workgroup LSD radix sort of up to THREADS * ITEMS keys held in
// registers and LDS (Sec. 4, Algorithms 4 and 5 at workgroup scale: per-digit
// counts, prefix sums, placement, with the paper's 8-bit digits).  Used for
// the short segments of a batched sort and for the small-array branch of the
// adaptive partition sort (Sec. 4.3, Algorithm 6).
//
// HBM sees one read and one write per key (and value): every pass ranks the
// keys stably with the wave64 lane-bucket rank of the device-wide pass,
// scatters them into LDS in digit order and reads them back in the striped
// order the next pass ranks in.
#pragma once

#include "common.hpp"

namespace evosort {

constexpr int kBlockLsdBits = 8;
constexpr int kBlockLsdBins = 1 << kBlockLsdBits;

// LDS of one workgroup.  The per-wave digit counters and lane buckets share
// storage with the staging area of one pass's scatter.  SPLIT stages keys
// and values one after the other (the area holds max(K, V) bytes per key
// instead of K + V), for a single workgroup that sorts many pairs.
template <int KB, int VB, int THREADS, int ITEMS, bool SPLIT>
struct BlockLsdLds {
    static constexpr int WAVES = THREADS / kWave;
    static constexpr int CAP = THREADS * ITEMS;
    static constexpr size_t BUCKET_OFFSET = ((size_t)WAVES * kBlockLsdBins * 4 + 15) & ~(size_t)15;
    static constexpr size_t HIST_BYTES = BUCKET_OFFSET + (size_t)WAVES * kBlockLsdBins * 8;
    static constexpr size_t ELEM_BYTES = SPLIT ? (KB > VB ? KB : VB) : (size_t)KB + VB;
    static constexpr size_t STAGE_BYTES = (size_t)CAP * ELEM_BYTES;
    // with SPLIT the values reuse the keys' area; otherwise they follow it
    static constexpr size_t VALS_OFFSET = SPLIT ? 0 : (size_t)CAP * KB;
    static constexpr size_t UNION_BYTES = HIST_BYTES > STAGE_BYTES ? HIST_BYTES : STAGE_BYTES;
    __attribute__((aligned(16))) unsigned char uni[UNION_BYTES];
    uint32_t wtot[WAVES];
    uint32_t job;
};

// Where one sort reads and writes.  Values are read from vals_in, or are the
// input positions begin + i when iota is set (argsort); keys are not written
// when skip_keys is set.
struct BlockLsdIo {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;
    void* vals_out;
    bool iota;
    bool skip_keys;
};

// Sorts keys [begin, begin + len) (len <= THREADS * ITEMS), stably, into the
// same range of the outputs; the outputs may be the inputs.  Wave w holds
// positions [w*64*ITEMS, (w+1)*64*ITEMS), item i lane-striped (position
// w*64*ITEMS + i*64 + lane), so ranking items in order and lanes in order
// visits positions in order: each pass is stable.  Ends with a barrier.
template <int KB, int VB, int THREADS, int ITEMS, bool SPLIT>
__device__ __forceinline__ void block_lsd_sort(const BlockLsdIo& io, const OrderMap<typename KeyWord<KB>::U>& om,
                                               BlockLsdLds<KB, VB, THREADS, ITEMS, SPLIT>& L, int64_t begin,
                                               uint32_t len)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using Lds = BlockLsdLds<KB, VB, THREADS, ITEMS, SPLIT>;
    constexpr int PASSES = KB;  // 8-bit digits
    constexpr int BINS = kBlockLsdBins;
    constexpr int WAVES = Lds::WAVES;
    constexpr int WAVE_KEYS = kWave * ITEMS;
    constexpr int BPT = (BINS + THREADS - 1) / THREADS;

    uint32_t* s_whist = reinterpret_cast<uint32_t*>(L.uni);
    uint64_t* s_bkt = reinterpret_cast<uint64_t*>(L.uni + Lds::BUCKET_OFFSET);
    U* s_keys = reinterpret_cast<U*>(L.uni);
    V* s_vals = reinterpret_cast<V*>(L.uni + Lds::VALS_OFFSET);

    const int lane = threadIdx.x & (kWave - 1);
    const int w = threadIdx.x / kWave;
    const uint32_t off0 = (uint32_t)(w * WAVE_KEYS + lane);
    const uint32_t wave_base = (uint32_t)(w * WAVE_KEYS);

    U k[ITEMS];
    V v[VB ? ITEMS : 1];
    {
        const U* kin = reinterpret_cast<const U*>(io.keys_in) + begin;
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t q = off0 + (uint32_t)(i * kWave);
            k[i] = q < len ? kin[q] : (U)0;
        }
        if constexpr (VB != 0) {
            const V* vin = reinterpret_cast<const V*>(io.vals_in) + begin;
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t q = off0 + (uint32_t)(i * kWave);
                v[i] = io.iota ? (V)(begin + q) : (q < len ? vin[q] : (V)0);
            }
        }
    }

    const uint64_t my_bit = 1ull << lane;
    for (int p = 0; p < PASSES; ++p) {
        const int shift = p * kBlockLsdBits;
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

        const bool last = p == PASSES - 1;
        // keys (and, unless split, values) through the staging area
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (rk[i] != 0xffffffffu) {
                s_keys[rk[i]] = k[i];
                if constexpr (VB != 0 && !SPLIT)
                    s_vals[rk[i]] = v[i];
            }
        }
        __syncthreads();
        if (last) {
            if (!io.skip_keys) {
                U* kout = reinterpret_cast<U*>(io.keys_out) + begin;
                for (uint32_t q = threadIdx.x; q < len; q += THREADS)
                    kout[q] = s_keys[q];
            }
            if constexpr (VB != 0 && !SPLIT) {
                V* vout = reinterpret_cast<V*>(io.vals_out) + begin;
                for (uint32_t q = threadIdx.x; q < len; q += THREADS)
                    vout[q] = s_vals[q];
            }
        } else {
#pragma unroll
            for (int i = 0; i < ITEMS; ++i) {
                const uint32_t q = off0 + (uint32_t)(i * kWave);
                if (q < len) {
                    k[i] = s_keys[q];
                    if constexpr (VB != 0 && !SPLIT)
                        v[i] = s_vals[q];
                }
            }
        }
        if constexpr (VB != 0 && SPLIT) {
            // values through the same area once the keys have left it
            __syncthreads();
#pragma unroll
            for (int i = 0; i < ITEMS; ++i)
                if (rk[i] != 0xffffffffu)
                    s_vals[rk[i]] = v[i];
            __syncthreads();
            if (last) {
                V* vout = reinterpret_cast<V*>(io.vals_out) + begin;
                for (uint32_t q = threadIdx.x; q < len; q += THREADS)
                    vout[q] = s_vals[q];
            } else {
#pragma unroll
                for (int i = 0; i < ITEMS; ++i) {
                    const uint32_t q = off0 + (uint32_t)(i * kWave);
                    if (q < len)
                        v[i] = s_vals[q];
                }
            }
        }
        __syncthreads();  // staging reads are done before the counters reuse it
    }
}

}  // namespace evosort
