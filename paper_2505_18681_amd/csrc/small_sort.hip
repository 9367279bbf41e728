// One-workgroup sort for arrays below the fallback threshold (the branch of
// Sec. 4.3, Algorithm 6 that hands small arrays to the platform's own sort).
//
// The whole array sits in LDS as records (order word, input position) and is
// sorted by a bitonic network (Batcher's construction).  Because positions are
// unique, every record is distinct and the network's result is the stable
// order.  Keys are written back from the order words (no second read of the
// input), values and indices from the recorded positions.
#include "common.hpp"
#include "small_sort.hpp"

namespace evosort {

namespace {

constexpr int kSmallThreads = 1024;

// 4-byte keys: one 64-bit word per record, order word above the position, so
// one integer comparison orders (key, position) pairs.
struct Rec4 {
    using Word = uint64_t;
    static constexpr Word kPad = ~0ull;
};

template <int KB>
struct SmallLds;
template <>
struct SmallLds<4> {
    uint64_t rec[kSmallCapacity4];
};
// 8-byte keys: order words and positions in two arrays, compared as pairs.
template <>
struct SmallLds<8> {
    uint64_t key[kSmallCapacity8];
    uint32_t pos[kSmallCapacity8];
};

template <int KB, int VB>
__global__ __launch_bounds__(kSmallThreads) void small_sort_kernel(SmallSortArgs a,
                                                                   OrderMap<typename KeyWord<KB>::U> om)
{
    using U = typename KeyWord<KB>::U;
    __shared__ SmallLds<KB> L;
    const int n = (int)a.n;
    int m = 1;
    while (m < n)
        m <<= 1;
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);

    // load and pad to a power of two
    for (int i = threadIdx.x; i < m; i += kSmallThreads) {
        if constexpr (KB == 4) {
            L.rec[i] = i < n ? ((uint64_t)om.to_order(keys_in[i]) << 32) | (uint32_t)i : Rec4::kPad;
        } else {
            L.key[i] = i < n ? om.to_order(keys_in[i]) : ~0ull;
            L.pos[i] = i < n ? (uint32_t)i : 0xffffffffu;
        }
    }
    __syncthreads();

    // bitonic network: stage k builds sorted runs of length k
    for (int k = 2; k <= m; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int t = threadIdx.x; t < (m >> 1); t += kSmallThreads) {
                const int lo = 2 * j * (t / j) + (t % j);
                const int hi = lo + j;
                const bool up = (lo & k) == 0;
                if constexpr (KB == 4) {
                    const uint64_t x = L.rec[lo], y = L.rec[hi];
                    if ((x > y) == up) {
                        L.rec[lo] = y;
                        L.rec[hi] = x;
                    }
                } else {
                    const uint64_t xk = L.key[lo], yk = L.key[hi];
                    const uint32_t xp = L.pos[lo], yp = L.pos[hi];
                    const bool gt = xk > yk || (xk == yk && xp > yp);
                    if (gt == up) {
                        L.key[lo] = yk;
                        L.key[hi] = xk;
                        L.pos[lo] = yp;
                        L.pos[hi] = xp;
                    }
                }
            }
            __syncthreads();
        }
    }

    // Each thread owns positions threadIdx.x + r * kSmallThreads.
    constexpr int R = (KB == 4 ? kSmallCapacity4 : kSmallCapacity8) / kSmallThreads;
    U kout[R];
    uint32_t src[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = threadIdx.x + r * kSmallThreads;
        if (i < n) {
            if constexpr (KB == 4) {
                kout[r] = om.from_order((U)(L.rec[i] >> 32));
                src[r] = (uint32_t)L.rec[i];
            } else {
                kout[r] = om.from_order(L.key[i]);
                src[r] = L.pos[i];
            }
        }
    }

    if constexpr (VB != 0) {
        using V = typename ValWord<VB>::T;
        if (a.mode == SMALL_MODE_PAIRS) {
            // Values may be sorted in place: every value is read and parked in
            // LDS (over the records, after a barrier) before any is written.
            const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
            V vin[R];
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = threadIdx.x + r * kSmallThreads;
                if (i < n)
                    vin[r] = vals_in[src[r]];
            }
            __syncthreads();
            V* park = reinterpret_cast<V*>(&L);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = threadIdx.x + r * kSmallThreads;
                if (i < n)
                    park[i] = vin[r];
            }
            __syncthreads();
            V* vals_out = reinterpret_cast<V*>(a.vals_out);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = threadIdx.x + r * kSmallThreads;
                if (i < n)
                    vals_out[i] = park[i];
            }
        } else {
            V* idx_out = reinterpret_cast<V*>(a.vals_out);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                const int i = threadIdx.x + r * kSmallThreads;
                if (i < n)
                    idx_out[i] = (V)src[r];
            }
        }
    }
    if (a.mode != SMALL_MODE_ARGSORT) {
        U* keys_out = reinterpret_cast<U*>(a.keys_out);
        // keys come from LDS, so writing over keys_in (in place) is safe once
        // every thread has loaded: the barriers above order that.
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = threadIdx.x + r * kSmallThreads;
            if (i < n)
                keys_out[i] = kout[r];
        }
    }
}

template <int KB, int VB>
hipError_t launch_t(const KeyDesc& kd, const SmallSortArgs& a, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL((small_sort_kernel<KB, VB>), dim3(1), dim3(kSmallThreads), 0, s, a, om);
    return hipGetLastError();
}

}  // namespace

int64_t small_sort_capacity(int key_bytes, int val_bytes)
{
    (void)val_bytes;
    return key_bytes == 4 ? kSmallCapacity4 : kSmallCapacity8;
}

hipError_t launch_small_sort(const KeyDesc& kd, int val_bytes, const SmallSortArgs& a, hipStream_t s)
{
    if (a.n > small_sort_capacity(kd.bytes, val_bytes))
        return hipErrorInvalidValue;
    if (kd.bytes == 4) {
        if (val_bytes == 0)
            return launch_t<4, 0>(kd, a, s);
        if (val_bytes == 4)
            return launch_t<4, 4>(kd, a, s);
        return launch_t<4, 8>(kd, a, s);
    }
    if (val_bytes == 0)
        return launch_t<8, 0>(kd, a, s);
    if (val_bytes == 4)
        return launch_t<8, 4>(kd, a, s);
    return launch_t<8, 8>(kd, a, s);
}

}  // namespace evosort
