// Bottom-up mergesort for gfx950 (Sec. 4, Algorithm 3, re-designed for one
// GPU).  The paper cuts the array into chunks of T_ins keys, insertion-sorts
// each chunk, then merges pairs of runs while the run length doubles.  Here:
//
//   merge_block_sort_kernel  one workgroup per block of T_ins * 2^m keys (as
//                            many as fit in LDS): every chunk of T_ins keys is
//                            put in order by rank counting (the parallel form
//                            of insertion sort: a key's place is the number of
//                            chunk keys before it in the stable order), then
//                            the chunks are merged pairwise inside LDS until
//                            the block is one run;
//   merge_partition_kernel   for every output tile of a merge round, a binary
//                            search along the tile's cross diagonal of the two
//                            runs (merge path) finds how many outputs come from
//                            the left run; ties go to the left run;
//   merge_round_kernel       one workgroup per output tile loads its two input
//                            slices into LDS, places every element by a binary
//                            search in the other slice, and writes the tile out
//                            coalesced.
//
// Stability: inside a block, records carry their position, so all records
// are distinct and every merge is exact.  Across blocks, the merge takes the
// left run's element first on equal keys.
#include "common.hpp"
#include "merge.hpp"

namespace evosort {

namespace {

constexpr int kMergeThreads = 256;

// ---------------------------------------------------------------- records --
template <int KB>
struct Rec;
template <>
struct Rec<4> {
    using W = uint64_t;  // order word << 32 | position in the block
    static __device__ __forceinline__ W make(uint32_t ord, uint32_t pos) { return ((uint64_t)ord << 32) | pos; }
    static __device__ __forceinline__ uint32_t ord(W r) { return (uint32_t)(r >> 32); }
    static __device__ __forceinline__ uint32_t pos(W r) { return (uint32_t)r; }
    static __device__ __forceinline__ bool less(W a, W b) { return a < b; }
};
template <>
struct Rec<8> {
    struct W {
        uint64_t ord;
        uint32_t pos;
        uint32_t pad;
    };
    static __device__ __forceinline__ W make(uint64_t ord, uint32_t pos) { return W{ord, pos, 0u}; }
    static __device__ __forceinline__ uint64_t ord(const W& r) { return r.ord; }
    static __device__ __forceinline__ uint32_t pos(const W& r) { return r.pos; }
    static __device__ __forceinline__ bool less(const W& a, const W& b)
    {
        return a.ord < b.ord || (a.ord == b.ord && a.pos < b.pos);
    }
};

template <int KB>
constexpr int block_cap()
{
    return KB == 4 ? 4096 : 2048;
}

// Number of records in buf[lo, hi) that are less than r.
template <int KB>
__device__ __forceinline__ int count_less(const typename Rec<KB>::W* buf, int lo, int hi, const typename Rec<KB>::W& r)
{
    int a = lo, b = hi;
    while (a < b) {
        const int mid = (a + b) >> 1;
        if (Rec<KB>::less(buf[mid], r))
            a = mid + 1;
        else
            b = mid;
    }
    return a - lo;
}

template <int KB, int VB>
__global__ __launch_bounds__(kMergeThreads) void merge_block_sort_kernel(MergeBlockArgs a,
                                                                         OrderMap<typename KeyWord<KB>::U> om,
                                                                         int t_ins, int block_keys)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using R = Rec<KB>;
    using W = typename R::W;
    constexpr int CAP = block_cap<KB>();
    __shared__ W buf[2][CAP];
    __shared__ V vpark[VB ? CAP : 1];

    const int64_t start = (int64_t)blockIdx.x * block_keys;
    const int64_t left = a.n - start;
    const int nb = left < block_keys ? (int)left : block_keys;
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);

    // Load the block.  Values are parked in LDS now, so that writing them
    // back over vals_in (in place) cannot race with reading them.
    for (int i = threadIdx.x; i < nb; i += kMergeThreads) {
        buf[0][i] = R::make(om.to_order(keys_in[start + i]), (uint32_t)i);
        if constexpr (VB != 0) {
            const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
            vpark[i] = a.iota ? (V)(start + i) : vals_in[start + i];
        }
    }
    __syncthreads();

    // Chunks of t_ins: place each record at (chunk start + number of smaller
    // records in its chunk).
    for (int i = threadIdx.x; i < nb; i += kMergeThreads) {
        const int c0 = (i / t_ins) * t_ins;
        const int c1 = c0 + t_ins < nb ? c0 + t_ins : nb;
        const W r = buf[0][i];
        int rank = 0;
        for (int j = c0; j < c1; ++j)
            rank += R::less(buf[0][j], r) ? 1 : 0;
        buf[1][c0 + rank] = r;
    }
    __syncthreads();

    // Pairwise merges inside the block, run length doubling from t_ins.
    int cur = 1;
    for (int L = t_ins; L < nb; L *= 2) {
        for (int i = threadIdx.x; i < nb; i += kMergeThreads) {
            const int s = (i / (2 * L)) * (2 * L);
            const int mid = s + L < nb ? s + L : nb;
            const int e = s + 2 * L < nb ? s + 2 * L : nb;
            const W r = buf[cur][i];
            int p;
            if (i < mid)
                p = (i - s) + count_less<KB>(buf[cur], mid, e, r);
            else
                p = (i - mid) + count_less<KB>(buf[cur], s, mid, r);
            buf[cur ^ 1][s + p] = r;
        }
        __syncthreads();
        cur ^= 1;
    }

    U* keys_out = reinterpret_cast<U*>(a.keys_out);
    for (int i = threadIdx.x; i < nb; i += kMergeThreads) {
        const W r = buf[cur][i];
        if (!a.skip_keys)
            keys_out[start + i] = om.from_order((U)R::ord(r));
        if constexpr (VB != 0) {
            V* vals_out = reinterpret_cast<V*>(a.vals_out);
            vals_out[start + i] = vpark[R::pos(r)];
        }
    }
}

// ---------------------------------------------------------- merge rounds --
struct RoundGeom {
    int64_t run;
    int64_t tpp;  // output tiles per pair of runs
    int64_t pairs;
    int tile_out;
};

__host__ __device__ inline RoundGeom round_geom(int64_t n, int64_t run, int tile_out)
{
    RoundGeom g;
    g.run = run;
    g.tile_out = tile_out;
    g.tpp = (2 * run + tile_out - 1) / tile_out;
    g.pairs = (n + 2 * run - 1) / (2 * run);
    return g;
}

template <int KB>
__global__ __launch_bounds__(kMergeThreads) void merge_partition_kernel(MergeRoundArgs a,
                                                                        OrderMap<typename KeyWord<KB>::U> om,
                                                                        RoundGeom g)
{
    using U = typename KeyWord<KB>::U;
    const int64_t idx = (int64_t)blockIdx.x * kMergeThreads + threadIdx.x;
    const int64_t total = g.pairs * (g.tpp + 1);
    if (idx >= total)
        return;
    const int64_t pair = idx / (g.tpp + 1);
    const int64_t t = idx % (g.tpp + 1);
    const int64_t s = pair * 2 * g.run;
    const int64_t na = a.n - s < g.run ? a.n - s : g.run;
    const int64_t rest = a.n - s - na;
    const int64_t nb = rest < g.run ? rest : g.run;
    const int64_t len = na + nb;
    const int64_t k = t * g.tile_out < len ? t * g.tile_out : len;
    const U* A = reinterpret_cast<const U*>(a.keys_in) + s;
    const U* B = A + na;
    // Outputs are A elements while A[i] <= B[k-i-1] (ties favour A).
    int64_t lo = k - nb > 0 ? k - nb : 0;
    int64_t hi = k < na ? k : na;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (om.to_order(A[mid]) <= om.to_order(B[k - mid - 1]))
            lo = mid + 1;
        else
            hi = mid;
    }
    a.parts[idx] = lo;
}

template <int KB, int VB, int TILE>
__global__ __launch_bounds__(kMergeThreads) void merge_round_kernel(MergeRoundArgs a,
                                                                    OrderMap<typename KeyWord<KB>::U> om,
                                                                    RoundGeom g)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    __shared__ U s_in[TILE];
    __shared__ U s_out[TILE];
    __shared__ V v_in[VB ? TILE : 1];
    __shared__ V v_out[VB ? TILE : 1];

    const int64_t pair = (int64_t)blockIdx.x / g.tpp;
    const int64_t t = (int64_t)blockIdx.x % g.tpp;
    const int64_t s = pair * 2 * g.run;
    const int64_t na = a.n - s < g.run ? a.n - s : g.run;
    const int64_t rest = a.n - s - na;
    const int64_t nb = rest < g.run ? rest : g.run;
    const int64_t len = na + nb;
    const int64_t k0 = t * TILE;
    if (k0 >= len)
        return;  // whole workgroup: tiles past the end of a short last pair
    const int64_t k1 = k0 + TILE < len ? k0 + TILE : len;
    const int64_t* parts = a.parts + pair * (g.tpp + 1);
    const int64_t a0 = parts[t], a1 = parts[t + 1];
    const int64_t b0 = k0 - a0, b1 = k1 - a1;
    // Merge-path splits are monotone and inside both runs; anything else
    // would mean a corrupted partition buffer, so the tile is left alone
    // rather than read out of range (the condition is uniform per workgroup).
    if (a0 < 0 || a1 < a0 || a1 > na || b0 < 0 || b1 < b0 || b1 > nb || k1 - k0 > TILE)
        return;
    const int ca = (int)(a1 - a0), cb = (int)(b1 - b0);
    const int cnt = ca + cb;

    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);
    const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
    for (int i = threadIdx.x; i < cnt; i += kMergeThreads) {
        const int64_t src = i < ca ? s + a0 + i : s + na + b0 + (i - ca);
        s_in[i] = om.to_order(keys_in[src]);
        if constexpr (VB != 0)
            v_in[i] = vals_in[src];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < cnt; i += kMergeThreads) {
        const U x = s_in[i];
        int p;
        if (i < ca) {
            // A element: after every B element strictly smaller
            int lo = ca, hi = cnt;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_in[mid] < x)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            p = i + (lo - ca);
        } else {
            // B element: after every A element smaller or equal
            int lo = 0, hi = ca;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (s_in[mid] <= x)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            p = (i - ca) + lo;
        }
        s_out[p] = x;
        if constexpr (VB != 0)
            v_out[p] = v_in[i];
    }
    __syncthreads();
    U* keys_out = reinterpret_cast<U*>(a.keys_out);
    V* vals_out = reinterpret_cast<V*>(a.vals_out);
    for (int i = threadIdx.x; i < cnt; i += kMergeThreads) {
        const int64_t dst = s + k0 + i;
        if (!a.skip_keys)
            keys_out[dst] = om.from_order(s_out[i]);
        if constexpr (VB != 0)
            vals_out[dst] = v_out[i];
    }
}

template <int KB>
constexpr int round_tile(int vb)
{
    return (KB + vb) <= 8 ? 4096 : 2048;
}

template <int KB, int VB>
hipError_t block_sort_t(const KeyDesc& kd, const MergePlan& mp, const MergeBlockArgs& a, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL((merge_block_sort_kernel<KB, VB>), dim3((unsigned)mp.blocks), dim3(kMergeThreads), 0, s, a,
                       om, (int)mp.t_ins, (int)mp.block_keys);
    return hipGetLastError();
}

template <int KB, int VB>
hipError_t round_t(const KeyDesc& kd, const MergePlan& mp, const MergeRoundArgs& a, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    constexpr int TILE = round_tile<KB>(VB);
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    const RoundGeom g = round_geom(a.n, a.run, TILE);
    const int64_t grid = g.pairs * g.tpp;
    if (grid > 0x7fffffffLL)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((merge_round_kernel<KB, VB, TILE>), dim3((unsigned)grid), dim3(kMergeThreads), 0, s, a, om,
                       g);
    (void)mp;
    return hipGetLastError();
}

}  // namespace

uint64_t merge_block_capacity(int kb, int vb)
{
    (void)vb;
    return kb == 4 ? (uint64_t)block_cap<4>() : (uint64_t)block_cap<8>();
}

static int round_tile_rt(int kb, int vb) { return (kb + vb) <= 8 ? 4096 : 2048; }

MergePlan merge_plan(int kb, int vb, int64_t n, uint32_t t_ins)
{
    MergePlan mp{};
    mp.kb = kb;
    mp.vb = vb;
    mp.n = n;
    mp.t_ins = t_ins;
    const uint64_t cap = merge_block_capacity(kb, vb);
    uint64_t block = t_ins;
    while (block * 2 <= cap)
        block *= 2;
    mp.block_keys = block;
    mp.block_run = block;
    mp.blocks = n > 0 ? ((uint64_t)n + block - 1) / block : 0;
    mp.tile_out = (uint32_t)round_tile_rt(kb, vb);
    uint32_t rounds = 0;
    uint64_t max_parts = 0;
    for (uint64_t run = block; run < (uint64_t)n; run *= 2) {
        ++rounds;
        const RoundGeom g = round_geom(n, (int64_t)run, (int)mp.tile_out);
        const uint64_t parts = (uint64_t)g.pairs * (uint64_t)(g.tpp + 1);
        if (parts > max_parts)
            max_parts = parts;
    }
    mp.rounds = rounds;
    mp.max_parts = max_parts;
    return mp;
}

uint64_t merge_round_parts(const MergePlan& mp, int64_t run)
{
    const RoundGeom g = round_geom(mp.n, run, (int)mp.tile_out);
    return (uint64_t)g.pairs * (uint64_t)(g.tpp + 1);
}

size_t merge_partition_bytes(const MergePlan& mp) { return (size_t)(mp.max_parts + 1) * sizeof(int64_t); }

hipError_t launch_merge_block_sort(const KeyDesc& kd, int vb, const MergePlan& mp, const MergeBlockArgs& a,
                                   hipStream_t s)
{
    if (mp.blocks == 0)
        return hipSuccess;
    if (mp.blocks > 0x7fffffffULL)
        return hipErrorInvalidValue;
    if (kd.bytes == 4) {
        if (vb == 0)
            return block_sort_t<4, 0>(kd, mp, a, s);
        if (vb == 4)
            return block_sort_t<4, 4>(kd, mp, a, s);
        return block_sort_t<4, 8>(kd, mp, a, s);
    }
    if (vb == 0)
        return block_sort_t<8, 0>(kd, mp, a, s);
    if (vb == 4)
        return block_sort_t<8, 4>(kd, mp, a, s);
    return block_sort_t<8, 8>(kd, mp, a, s);
}

hipError_t launch_merge_partition(const KeyDesc& kd, const MergePlan& mp, const MergeRoundArgs& a, hipStream_t s)
{
    const RoundGeom g = round_geom(a.n, a.run, (int)mp.tile_out);
    const int64_t total = g.pairs * (g.tpp + 1);
    if ((uint64_t)total > mp.max_parts + 1)
        return hipErrorInvalidValue;  // partition buffer sized for a different round shape
    const int64_t grid = (total + kMergeThreads - 1) / kMergeThreads;
    if (grid == 0)
        return hipSuccess;
    if (kd.bytes == 4) {
        OrderMap<uint32_t> om{(uint32_t)kd.flip, (uint32_t)kd.neg, (uint32_t)kd.desc};
        hipLaunchKernelGGL((merge_partition_kernel<4>), dim3((unsigned)grid), dim3(kMergeThreads), 0, s, a, om, g);
    } else {
        OrderMap<uint64_t> om{kd.flip, kd.neg, kd.desc};
        hipLaunchKernelGGL((merge_partition_kernel<8>), dim3((unsigned)grid), dim3(kMergeThreads), 0, s, a, om, g);
    }
    return hipGetLastError();
}

hipError_t launch_merge_round(const KeyDesc& kd, int vb, const MergePlan& mp, const MergeRoundArgs& a,
                              hipStream_t s)
{
    if (a.n == 0)
        return hipSuccess;
    if (kd.bytes == 4) {
        if (vb == 0)
            return round_t<4, 0>(kd, mp, a, s);
        if (vb == 4)
            return round_t<4, 4>(kd, mp, a, s);
        return round_t<4, 8>(kd, mp, a, s);
    }
    if (vb == 0)
        return round_t<8, 0>(kd, mp, a, s);
    if (vb == 4)
        return round_t<8, 4>(kd, mp, a, s);
    return round_t<8, 8>(kd, mp, a, s);
}

hipError_t run_merge_sort(const MergePlan& mp, const MergeBuffers& b, const MergeLaunch& ml)
{
    const int R = (int)mp.rounds;
    const bool argsort = b.iota;
    // Destination of stage st (0 = block sort, 1..R = merge rounds); the last
    // stage writes the outputs.
    auto key_dst = [&](int st) -> void* {
        if (argsort)
            return (st & 1) ? b.keys_tmp2 : b.keys_tmp;
        return ((R - st) & 1) ? b.keys_tmp : b.keys_out;
    };
    auto val_dst = [&](int st) -> void* {
        if (!mp.vb)
            return nullptr;
        return ((R - st) & 1) ? b.vals_tmp : b.vals_out;
    };
    MergeBlockArgs ba{};
    ba.keys_in = b.keys_in;
    ba.keys_out = key_dst(0);
    ba.vals_in = b.vals_in;
    ba.vals_out = val_dst(0);
    ba.n = mp.n;
    ba.iota = argsort;
    ba.skip_keys = argsort && R == 0;
    hipError_t e = ml.block_sort(ba);
    if (e != hipSuccess)
        return e;
    int64_t run = (int64_t)mp.block_run;
    for (int st = 1; st <= R; ++st, run *= 2) {
        MergeRoundArgs ra{};
        ra.keys_in = key_dst(st - 1);
        ra.keys_out = key_dst(st);
        ra.vals_in = val_dst(st - 1);
        ra.vals_out = val_dst(st);
        ra.n = mp.n;
        ra.run = run;
        ra.parts = b.parts;
        ra.skip_keys = argsort && st == R;
        e = ml.partition(ra);
        if (e != hipSuccess)
            return e;
        e = ml.merge(ra);
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

}  // namespace evosort
