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
//                            slices into LDS, merges them, and writes the tile
//                            out coalesced.
//
// Every merge inside LDS (the block's levels and a round's tile) is split the
// same way: each thread owns a run of consecutive outputs and finds where its
// run starts on both inputs by one merge-path search; it then loads that many
// elements of both inputs from there into registers and keeps the smallest
// with a bitonic merging network (merge_window), or, where a block level's
// pairs of runs are not a multiple of the thread's run, merges sequentially
// with both heads in registers (merge_run).  LDS arrays are padded by one
// element every 16, so that the threads' runs start in different banks.
//
// Stability: with values, block records carry their position, so all records
// are distinct and every merge is exact; keys-only blocks rank chunk mates by
// (key, index) and merge left-first, which leaves equal keys in input order.
// Across blocks, the merge takes the left run's element first on equal keys.
#include "common.hpp"
#include "merge.hpp"

namespace evosort {

namespace {

constexpr int kPartitionThreads = 256;  // partition kernel
constexpr int kRoundThreads = 512;      // round kernel
constexpr int kBlockSortThreads = 512;  // block sort

// LDS index of element p of a padded array: one spare element every 16.
__device__ __forceinline__ int pad16(int p) { return p + (p >> 4); }
constexpr int padded16(int n) { return n + (n >> 4) + 1; }

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
    // above every record (positions are below 2^32 - 1)
    static __device__ __forceinline__ W top() { return ~0ull; }
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
    static __device__ __forceinline__ W top() { return W{~0ull, 0xffffffffu, 0u}; }
};

// Records of the block sort.  Keys-only blocks hold bare order words: a
// chunk ranks a key against its chunk mates by (word, position), positions
// being the records' indices, and the merges take the left run's record on
// equal words, so the block is stable without storing positions.  With values
// (or indices) a record also carries the key's position in the block, which
// tells where its value is parked.
template <int KB, int VB>
struct BlockRec {
    using R = Rec<KB>;
    using W = typename R::W;
    static constexpr bool kBare = false;
    static __device__ __forceinline__ W make(typename KeyWord<KB>::U ord, uint32_t pos) { return R::make(ord, pos); }
    static __device__ __forceinline__ typename KeyWord<KB>::U ord(const W& r) { return (typename KeyWord<KB>::U)R::ord(r); }
    static __device__ __forceinline__ uint32_t pos(const W& r) { return R::pos(r); }
    static __device__ __forceinline__ bool less(const W& a, const W& b) { return R::less(a, b); }
    // x (at index jx) comes before y (at index iy) in the stable order
    static __device__ __forceinline__ bool before(const W& x, int, const W& y, int) { return R::less(x, y); }
    static __device__ __forceinline__ W top() { return R::top(); }
};
template <int KB>
struct BlockRec<KB, 0> {
    using W = typename KeyWord<KB>::U;
    static constexpr bool kBare = true;
    static __device__ __forceinline__ W make(W ord, uint32_t) { return ord; }
    static __device__ __forceinline__ W ord(W r) { return r; }
    static __device__ __forceinline__ bool less(W a, W b) { return a < b; }
    static __device__ __forceinline__ bool before(W x, int jx, W y, int iy) { return x < y || (x == y && jx < iy); }
    static __device__ __forceinline__ W top() { return ~(W)0; }
};

// A key with its index in a round's input slice.
template <typename U>
struct KeyIdx;
template <>
struct KeyIdx<uint32_t> {
    uint64_t w;  // key << 32 | index
    static __device__ __forceinline__ KeyIdx make(uint32_t key, uint32_t idx) { return {((uint64_t)key << 32) | idx}; }
    static __device__ __forceinline__ uint32_t key(const KeyIdx& r) { return (uint32_t)(r.w >> 32); }
    static __device__ __forceinline__ uint32_t idx(const KeyIdx& r) { return (uint32_t)r.w; }
    static __device__ __forceinline__ bool less(const KeyIdx& a, const KeyIdx& b) { return a.w < b.w; }
    static __device__ __forceinline__ KeyIdx top() { return {~0ull}; }
};
template <>
struct KeyIdx<uint64_t> {
    uint64_t k;
    uint32_t i;
    static __device__ __forceinline__ KeyIdx make(uint64_t key, uint32_t idx) { return {key, idx}; }
    static __device__ __forceinline__ uint64_t key(const KeyIdx& r) { return r.k; }
    static __device__ __forceinline__ uint32_t idx(const KeyIdx& r) { return r.i; }
    static __device__ __forceinline__ bool less(const KeyIdx& a, const KeyIdx& b)
    {
        return a.k < b.k || (a.k == b.k && a.i < b.i);
    }
    static __device__ __forceinline__ KeyIdx top() { return {~0ull, 0xffffffffu}; }
};

// Keys per block-sort workgroup: 4096, or 2048 for 16-byte records.
template <int KB, int VB>
constexpr int block_cap()
{
    return KB == 8 && VB != 0 ? 2048 : 4096;
}

// Merges the sorted runs A = src[a0, a0 + na) and B = src[b0, b0 + nb)
// (padded indices) and writes outputs [k, k_end) of the merge to
// dst[d0 + k, d0 + k_end).  `less` is the merge order with ties already
// decided: an A element goes first iff !less(B element, A element).  Returns
// nothing; every thread calls it for its own output run.
template <typename T, typename Less, typename Emit>
__device__ __forceinline__ void merge_run(const T* src, int a0, int na, int b0, int nb, int k, int k_end,
                                          const T& top, Less less, Emit emit)
{
    // merge path: i = A elements among the first k outputs
    int lo = k - nb > 0 ? k - nb : 0;
    int hi = k < na ? k : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (!less(src[pad16(b0 + k - 1 - mid)], src[pad16(a0 + mid)]))
            lo = mid + 1;  // A[mid] goes before B[k-1-mid]
        else
            hi = mid;
    }
    int i = lo, j = k - lo;
    T ha = i < na ? src[pad16(a0 + i)] : top;
    T hb = j < nb ? src[pad16(b0 + j)] : top;
    for (int o = k; o < k_end; ++o) {
        // branch-free step: emit the smaller head, refill it with one read
        const bool take_a = j >= nb || (i < na && !less(hb, ha));
        emit(o, take_a ? ha : hb, take_a ? a0 + i : b0 + j);
        i += take_a ? 1 : 0;
        j += take_a ? 0 : 1;
        const int next = take_a ? a0 + i : b0 + j;
        const bool more = take_a ? i < na : j < nb;
        const T x = src[pad16(more ? next : a0)];  // a0 is always a valid index
        const T nx = more ? x : top;
        ha = take_a ? nx : ha;
        hb = take_a ? hb : nx;
    }
}

// Outputs [k, k_end) (at most PER of them) of the merge of the sorted runs A
// (indices a0 .. a0 + na - 1) and B (b0 .. b0 + nb - 1), read with load(index),
// with the same tie rule as merge_run.  After the merge-path search the thread
// loads PER elements of each run from where its outputs start (independent
// reads), and keeps the PER smallest of them: for ascending x and y,
// min(x[q], y[PER-1-q]) are the PER smallest and form a bitonic sequence, which
// a bitonic merging network puts in order.  All in registers, no branches.
template <int PER, typename T, typename Load, typename Less, typename Emit>
__device__ __forceinline__ void merge_window(Load load, int a0, int na, int b0, int nb, int k, int k_end,
                                             const T& top, Less less, Emit emit)
{
    static_assert(PER >= 2 && (PER & (PER - 1)) == 0, "a power of two");
    int lo = k - nb > 0 ? k - nb : 0;
    int hi = k < na ? k : na;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (!less(load(b0 + k - 1 - mid), load(a0 + mid)))
            lo = mid + 1;  // A[mid] goes before B[k-1-mid]
        else
            hi = mid;
    }
    const int i0 = lo, j0 = k - lo;
    T x[PER], y[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        x[q] = i0 + q < na ? load(a0 + i0 + q) : top;
        y[q] = j0 + q < nb ? load(b0 + j0 + q) : top;
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const T v = y[PER - 1 - q];
        x[q] = less(v, x[q]) ? v : x[q];  // A's element on ties
    }
#pragma unroll
    for (int st = PER / 2; st >= 1; st >>= 1) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if ((q & st) == 0) {
                const T u = x[q], v = x[q + st];
                const bool sw = less(v, u);
                x[q] = sw ? v : u;
                x[q + st] = sw ? u : v;
            }
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (k + q < k_end)
            emit(k + q, x[q]);
}

template <int KB, int VB>
__global__ __launch_bounds__(kBlockSortThreads) void merge_block_sort_kernel(MergeBlockArgs a,
                                                                             OrderMap<typename KeyWord<KB>::U> om,
                                                                             int t_ins, int block_keys)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using R = BlockRec<KB, VB>;
    using W = typename R::W;
    constexpr int CAP = block_cap<KB, VB>();
    __shared__ W buf[2][padded16(CAP)];
    __shared__ V vpark[VB ? CAP : 1];

    const int64_t start = (int64_t)blockIdx.x * block_keys;
    const int64_t left = a.n - start;
    const int nb = left < block_keys ? (int)left : block_keys;
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);

    // Load the block.  Values are parked in LDS now, so that writing them
    // back over vals_in (in place) cannot race with reading them.  A thread's
    // loads are all issued before any of them is waited for.
    constexpr int LOADS = CAP / kBlockSortThreads;
    {
        U kr[LOADS];
        V vr[VB ? LOADS : 1];
        const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const int i = threadIdx.x + q * kBlockSortThreads;
            if (i < nb) {
                kr[q] = keys_in[start + i];
                if constexpr (VB != 0)
                    vr[q] = a.iota ? (V)(start + i) : vals_in[start + i];
            }
        }
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const int i = threadIdx.x + q * kBlockSortThreads;
            if (i < nb) {
                buf[0][pad16(i)] = R::make(om.to_order(kr[q]), (uint32_t)i);
                if constexpr (VB != 0)
                    vpark[i] = vr[q];
            }
        }
    }
    __syncthreads();

    constexpr int PER = CAP / kBlockSortThreads;
    if (t_ins == PER && nb == CAP) {
        // Chunks of exactly one thread's PER records (a full block): the
        // thread puts its chunk in order in registers with a bitonic sorting
        // network.  Records compare by (word, position) -- positions are
        // distinct, or with bare words equal records are identical -- so the
        // network's order is the stable order insertion sort gives.
        W x[PER];
        const int c0 = threadIdx.x * PER;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            x[q] = buf[0][pad16(c0 + q)];
#pragma unroll
        for (int size = 2; size <= PER; size *= 2) {
#pragma unroll
            for (int st = size / 2; st >= 1; st /= 2) {
#pragma unroll
                for (int q = 0; q < PER; ++q) {
                    const int pq = q ^ st;
                    if (pq > q) {
                        const bool up = (q & size) == 0;
                        const bool sw = up ? R::before(x[pq], c0 + pq, x[q], c0 + q)
                                           : R::before(x[q], c0 + q, x[pq], c0 + pq);
                        const W lo = sw ? x[pq] : x[q];
                        const W hi = sw ? x[q] : x[pq];
                        x[q] = lo;
                        x[pq] = hi;
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q)
            buf[1][pad16(c0 + q)] = x[q];
    } else {
        // Chunks of t_ins: place each record at (chunk start + number of
        // smaller records in its chunk).
        for (int i = threadIdx.x; i < nb; i += kBlockSortThreads) {
            const int c0 = (i / t_ins) * t_ins;
            const int c1 = c0 + t_ins < nb ? c0 + t_ins : nb;
            const W r = buf[0][pad16(i)];
            int rank = 0;
            for (int j = c0; j < c1; ++j)
                rank += R::before(buf[0][pad16(j)], j, r, i) ? 1 : 0;
            buf[1][pad16(c0 + rank)] = r;
        }
    }
    __syncthreads();

    // Pairwise merges inside the block, run length doubling from t_ins; on
    // equal records the left run's goes first.  Thread t owns outputs
    // [t*PER, (t+1)*PER) of every level.
    const auto less = [](const W& x, const W& y) { return R::less(x, y); };
    int cur = 1;
    for (int L = t_ins; L < nb; L *= 2) {
        const W* src = buf[cur];
        W* dst = buf[cur ^ 1];
        int o = threadIdx.x * PER;
        const int o_end = o + PER < nb ? o + PER : nb;
        if ((2 * L) % PER == 0) {
            // a thread's outputs lie in one pair of runs
            if (o < o_end) {
                const int s = (o / (2 * L)) * (2 * L);
                const int mid = s + L < nb ? s + L : nb;
                const int e = s + 2 * L < nb ? s + 2 * L : nb;
                merge_window<PER, W>([&](int i) { return src[pad16(i)]; }, s, mid - s, mid, e - mid, o - s,
                                     o_end - s, R::top(), less, [&](int q, const W& r) { dst[pad16(s + q)] = r; });
            }
        } else {
            while (o < o_end) {  // the thread's outputs may span pairs of runs
                const int s = (o / (2 * L)) * (2 * L);
                const int mid = s + L < nb ? s + L : nb;
                const int e = s + 2 * L < nb ? s + 2 * L : nb;
                const int stop = o_end < e ? o_end : e;
                merge_run<W>(src, s, mid - s, mid, e - mid, o - s, stop - s, R::top(), less,
                             [&](int q, const W& r, int) { dst[pad16(s + q)] = r; });
                o = stop;
            }
        }
        __syncthreads();
        cur ^= 1;
    }

    U* keys_out = reinterpret_cast<U*>(a.keys_out);
    for (int i = threadIdx.x; i < nb; i += kBlockSortThreads) {
        const W r = buf[cur][pad16(i)];
        if (!a.skip_keys)
            keys_out[start + i] = om.from_order((U)R::ord(r));
        if constexpr (!R::kBare) {
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
__global__ __launch_bounds__(kPartitionThreads) void merge_partition_kernel(MergeRoundArgs a,
                                                                        OrderMap<typename KeyWord<KB>::U> om,
                                                                        RoundGeom g)
{
    using U = typename KeyWord<KB>::U;
    const int64_t idx = (int64_t)blockIdx.x * kPartitionThreads + threadIdx.x;
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
__global__ __launch_bounds__(kRoundThreads) void merge_round_kernel(MergeRoundArgs a,
                                                                    OrderMap<typename KeyWord<KB>::U> om,
                                                                    RoundGeom g)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    constexpr int PER = TILE / kRoundThreads;
    __shared__ U s_in[padded16(TILE)];
    __shared__ U s_out[padded16(TILE)];
    __shared__ V v_in[VB ? TILE : 1];
    __shared__ V v_out[VB ? padded16(TILE) : 1];

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

    // the tile's A slice, then its B slice; a thread's loads are all issued
    // before any of them is waited for
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);
    const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
    {
        U kr[PER];
        V vr[VB ? PER : 1];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = threadIdx.x + q * kRoundThreads;
            if (i < cnt) {
                const int64_t src = i < ca ? s + a0 + i : s + na + b0 + (i - ca);
                kr[q] = keys_in[src];
                if constexpr (VB != 0)
                    vr[q] = vals_in[src];
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i = threadIdx.x + q * kRoundThreads;
            if (i < cnt) {
                s_in[pad16(i)] = om.to_order(kr[q]);
                if constexpr (VB != 0)
                    v_in[i] = vr[q];
            }
        }
    }
    __syncthreads();
    {
        const int o = threadIdx.x * PER;
        const int o_end = o + PER < cnt ? o + PER : cnt;
        if (o < o_end) {
            // ties favour the A run: an A element goes first unless B's is smaller
            if constexpr (VB == 0) {
                merge_window<PER, U>([&](int i) { return s_in[pad16(i)]; }, 0, ca, ca, cb, o, o_end, (U)~(U)0,
                                     [](U x, U y) { return x < y; }, [&](int q, U key) { s_out[pad16(q)] = key; });
            } else {
                // (key, slice index) pairs: A's indices are below B's, so the
                // order of the pairs is the merge order with A first on ties,
                // and the index finds the value
                using KI = KeyIdx<U>;
                merge_window<PER, KI>([&](int i) { return KI::make(s_in[pad16(i)], (uint32_t)i); }, 0, ca, ca, cb, o,
                                      o_end, KI::top(), [](const KI& x, const KI& y) { return KI::less(x, y); },
                                      [&](int q, const KI& r) {
                                          s_out[pad16(q)] = KI::key(r);
                                          v_out[pad16(q)] = v_in[KI::idx(r)];
                                      });
            }
        }
    }
    __syncthreads();
    U* keys_out = reinterpret_cast<U*>(a.keys_out);
    V* vals_out = reinterpret_cast<V*>(a.vals_out);
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int i = threadIdx.x + q * kRoundThreads;
        if (i < cnt) {
            const int64_t dst = s + k0 + i;
            if (!a.skip_keys)
                keys_out[dst] = om.from_order(s_out[pad16(i)]);
            if constexpr (VB != 0)
                vals_out[dst] = v_out[pad16(i)];
        }
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
    if (mp.block_keys > (uint64_t)block_cap<KB, VB>() || mp.block_keys == 0)
        return hipErrorInvalidValue;  // a plan made for another value width
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    hipLaunchKernelGGL((merge_block_sort_kernel<KB, VB>), dim3((unsigned)mp.blocks), dim3(kBlockSortThreads), 0, s, a,
                       om, (int)mp.t_ins, (int)mp.block_keys);
    return hipGetLastError();
}

template <int KB, int VB>
hipError_t round_t(const KeyDesc& kd, const MergePlan& mp, const MergeRoundArgs& a, hipStream_t s)
{
    using U = typename KeyWord<KB>::U;
    constexpr int TILE = round_tile<KB>(VB);
    if (mp.tile_out != (uint32_t)TILE)
        return hipErrorInvalidValue;  // the partition was cut for another tile
    OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};
    const RoundGeom g = round_geom(a.n, a.run, TILE);
    const int64_t grid = g.pairs * g.tpp;
    if (grid > 0x7fffffffLL)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL((merge_round_kernel<KB, VB, TILE>), dim3((unsigned)grid), dim3(kRoundThreads), 0, s, a, om,
                       g);
    return hipGetLastError();
}

}  // namespace

uint64_t merge_block_capacity(int kb, int vb)
{
    if (kb == 4)
        return vb ? (uint64_t)block_cap<4, 4>() : (uint64_t)block_cap<4, 0>();
    return vb ? (uint64_t)block_cap<8, 4>() : (uint64_t)block_cap<8, 0>();
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
    const int64_t grid = (total + kPartitionThreads - 1) / kPartitionThreads;
    if (grid == 0)
        return hipSuccess;
    if (kd.bytes == 4) {
        OrderMap<uint32_t> om{(uint32_t)kd.flip, (uint32_t)kd.neg, (uint32_t)kd.desc};
        hipLaunchKernelGGL((merge_partition_kernel<4>), dim3((unsigned)grid), dim3(kPartitionThreads), 0, s, a, om, g);
    } else {
        OrderMap<uint64_t> om{kd.flip, kd.neg, kd.desc};
        hipLaunchKernelGGL((merge_partition_kernel<8>), dim3((unsigned)grid), dim3(kPartitionThreads), 0, s, a, om, g);
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
