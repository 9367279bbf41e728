// Bottom-up mergesort for gfx950 (Sec. 4, Algorithm 3, re-designed for one
// GPU).  The paper cuts the array into chunks of T_ins keys, insertion-sorts
// each chunk, then merges pairs of runs while the run length doubles.  Here:
//
//   merge_block_sort_kernel  one workgroup per block of T_ins * 2^m keys (as
//                            many as fit in LDS), 8 keys per thread: every
//                            chunk of T_ins keys is put in order by rank
//                            counting (the parallel form of insertion sort: a
//                            key's place is the number of chunk keys before it
//                            in the stable order), then the chunks are merged
//                            pairwise inside LDS until the block is one run.
//                            A full block with T_ins dividing 8 takes the
//                            register path instead: each thread sorts its 8
//                            keys, the wave merges them up to runs of 512 with
//                            bitonic merges across lanes (DPP and swizzles),
//                            and each later level is merged in LDS one wave
//                            per 512 outputs (wave_lds_merge);
//   merge_partition_kernel   for every output tile of a merge round, a binary
//                            search along the tile's cross diagonal of the two
//                            runs (merge path) finds how many outputs come from
//                            the left run; ties go to the left run;
//   merge_round_kernel       one workgroup per output tile loads its two input
//                            slices into LDS, merges them, and writes the tile
//                            out coalesced.
//
// A round's tile, and the block levels off the register path, are merged in
// LDS the same way: each thread owns a run of consecutive outputs and finds
// where its run starts on both inputs by one merge-path search; it then loads
// that many elements of both inputs from there into registers and keeps the
// smallest with a bitonic merging network (merge_window), or, where a block
// level's pairs of runs are not a multiple of the thread's run, merges
// sequentially with both heads in registers (merge_run).  LDS arrays are
// padded by one element every 16, so that the threads' runs start in
// different banks.
//
// Stability: with values, block records carry their position, so all records
// are distinct and every merge is exact; keys-only blocks rank chunk mates by
// (key, index) and merge left-first, which leaves equal keys in input order.
// Across blocks, the merge takes the left run's element first on equal keys.
#include "common.hpp"
#include "merge.hpp"

namespace evosort {

namespace {

constexpr int kPartitionThreads = 64;   // partition kernel: one wave per workgroup, spread over every CU
constexpr int kRoundThreads = 512;      // round kernel
constexpr int kBlockPer = 8;            // block sort: records per thread

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

// c ? a : b, field by field for the 16-byte records: a select of the whole
// aggregate can be lowered through private (scratch) memory.
template <typename T>
__device__ __forceinline__ T pick(bool c, const T& a, const T& b)
{
    return c ? a : b;
}
__device__ __forceinline__ Rec<8>::W pick(bool c, const Rec<8>::W& a, const Rec<8>::W& b)
{
    return Rec<8>::W{c ? a.ord : b.ord, c ? a.pos : b.pos, 0u};
}
__device__ __forceinline__ KeyIdx<uint64_t> pick(bool c, const KeyIdx<uint64_t>& a, const KeyIdx<uint64_t>& b)
{
    return KeyIdx<uint64_t>{c ? a.k : b.k, c ? a.i : b.i};
}

// (a, b) <- (the smaller, the larger) under `less`; records that `less`
// does not order are identical.  Bare 32-bit words take min and max.
template <typename W, typename Less>
__device__ __forceinline__ void order2(W& a, W& b, Less less)
{
    const bool sw = less(b, a);
    const W lo = pick(sw, b, a), hi = pick(sw, a, b);
    a = lo;
    b = hi;
}
template <typename Less>
__device__ __forceinline__ void order2(uint32_t& a, uint32_t& b, Less)
{
    const uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
    a = lo;
    b = hi;
}

// Keys per block-sort workgroup: 4096, or 2048 for 16-byte records; the
// workgroup has one thread per kBlockPer of them.
template <int KB, int VB>
constexpr int block_cap()
{
    return KB == 8 && VB != 0 ? 2048 : 4096;
}
template <int KB, int VB>
constexpr int block_threads()
{
    return block_cap<KB, VB>() / kBlockPer;
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
        emit(o, pick(take_a, ha, hb), take_a ? a0 + i : b0 + j);
        i += take_a ? 1 : 0;
        j += take_a ? 0 : 1;
        const int next = take_a ? a0 + i : b0 + j;
        const bool more = take_a ? i < na : j < nb;
        const T x = src[pad16(more ? next : a0)];  // a0 is always a valid index
        const T nx = pick(more, x, top);
        ha = pick(take_a, nx, ha);
        hb = pick(take_a, hb, nx);
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
        x[q] = pick(less(v, x[q]), v, x[q]);  // A's element on ties
    }
#pragma unroll
    for (int st = PER / 2; st >= 1; st >>= 1) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            if ((q & st) == 0)
                order2(x[q], x[q + st], less);
        }
    }
#pragma unroll
    for (int q = 0; q < PER; ++q)
        if (k + q < k_end)
            emit(k + q, x[q]);
}

// --------------------------------------------------------- wave exchanges --
// The 32-bit register v of lane (lane ^ M) of the wave.  Masks inside a row
// of 16 lanes are DPP moves (no LDS pipe); 16 and 31 swizzle inside 32 lanes;
// 32 and 63 go through ds_bpermute.
template <int M>
__device__ __forceinline__ uint32_t lane_xor32(uint32_t v, int lane)
{
    const int s = (int)v;
    if constexpr (M == 1)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0xB1, 0xF, 0xF, true);  // quad_perm [1,0,3,2]
    else if constexpr (M == 2)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x4E, 0xF, 0xF, true);  // quad_perm [2,3,0,1]
    else if constexpr (M == 3)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x1B, 0xF, 0xF, true);  // quad_perm [3,2,1,0]
    else if constexpr (M == 7)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x141, 0xF, 0xF, true);  // row_half_mirror
    else if constexpr (M == 15)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x140, 0xF, 0xF, true);  // row_mirror
    else if constexpr (M == 8)
        return (uint32_t)__builtin_amdgcn_mov_dpp(s, 0x128, 0xF, 0xF, true);  // row_ror:8
    else if constexpr (M == 4)
        return lane_xor32<3>(lane_xor32<7>(v, lane), lane);  // (l ^ 7) ^ 3
    else if constexpr (M == 16 || M == 31)
        return (uint32_t)__builtin_amdgcn_ds_swizzle(s, (M << 10) | 0x1F);  // bit mode: l ^ M in 32 lanes
    else {
        static_assert(M == 32 || M == 63, "mask not provided");
        return (uint32_t)__builtin_amdgcn_ds_bpermute((lane ^ M) << 2, s);
    }
}

template <int M>
__device__ __forceinline__ uint32_t lane_xor(uint32_t v, int lane)
{
    return lane_xor32<M>(v, lane);
}
template <int M>
__device__ __forceinline__ uint64_t lane_xor(uint64_t v, int lane)
{
    const uint32_t lo = lane_xor32<M>((uint32_t)v, lane);
    const uint32_t hi = lane_xor32<M>((uint32_t)(v >> 32), lane);
    return ((uint64_t)hi << 32) | lo;
}
template <int M>
__device__ __forceinline__ Rec<8>::W lane_xor(const Rec<8>::W& v, int lane)
{
    return Rec<8>::W{lane_xor<M>(v.ord, lane), lane_xor32<M>(v.pos, lane), 0u};
}

// Half-cleaner steps of a bitonic merge across lanes: every register of lane
// l meets the same register of lane l ^ M, for M = M0, M0 / 2, ..., 1; the
// lower lane keeps the smaller.
template <int M, int N, typename W, typename Less>
__device__ __forceinline__ void half_clean_lanes(W (&x)[N], int lane, Less less)
{
    if constexpr (M >= 1) {
        // the lower lane takes y when it is smaller, the upper when it is not
        const bool high = (lane & M) != 0;
#pragma unroll
        for (int q = 0; q < N; ++q) {
            const W y = lane_xor<M>(x[q], lane);
            x[q] = pick(less(y, x[q]) != high, y, x[q]);
        }
        half_clean_lanes<M / 2>(x, lane, less);
    }
}

// Merge levels of run length L = PER, 2 PER, ..., 32 PER inside one wave,
// in registers: lane l holds records [l PER, (l + 1) PER) of the wave's
// 64 PER, each lane's PER in order on entry, all 64 PER in order on exit.  A
// level pairs runs of L records (L / PER lanes) and merges each pair with a
// bitonic merge: every record of the left run meets its mirror image in the
// right run, then half-cleaners at distances L/2 down to 1 sort both halves.
// Records compare by `less`, under which no two distinct records are equal,
// so the result is the one unique order the LDS merges would give.
template <int PER, int L, typename W, typename Less>
__device__ __forceinline__ void wave_merge_levels(W (&x)[PER], int lane, Less less)
{
    if constexpr (L < 64 * PER) {
        constexpr int G = 2 * L / PER;  // lanes holding one pair of runs
        const bool high = (lane & (G / 2)) != 0;
        W y[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q)
            y[q] = lane_xor<G - 1>(x[PER - 1 - q], lane);
#pragma unroll
        for (int q = 0; q < PER; ++q)
            x[q] = pick(less(y[q], x[q]) != high, y[q], x[q]);
        half_clean_lanes<L / 2 / PER>(x, lane, less);  // distances L/2 .. PER: across lanes
#pragma unroll
        for (int st = PER / 2; st >= 1; st >>= 1) {
#pragma unroll
            for (int q = 0; q < PER; ++q)
                if ((q & st) == 0)
                    order2(x[q], x[q + st], less);
        }
        wave_merge_levels<PER, 2 * L>(x, lane, less);
    }
}

// Number of A elements among the first k outputs of the merge of the sorted
// runs A = src[a0, a0 + L) and B = src[b0, b0 + L) (merge path, A first on
// ties), found by the whole wave: each round the 64 lanes test 64 evenly
// spaced candidates at once and a ballot keeps the interval between the last
// that passes and the first that fails, so runs of up to 4096 take two
// rounds.  Wave-uniform arguments; every lane returns the same value.
template <typename W, typename Less>
__device__ __forceinline__ int wave_merge_path(const W* src, int a0, int b0, int L, int k, int lane, Less less)
{
    int lo = k - L > 0 ? k - L : 0;
    int hi = k < L ? k : L;
    while (lo < hi) {
        const int step = (hi - lo + 63) >> 6;
        const int c = lo + (lane + 1) * step;
        // A[c - 1] goes before B[k - c]: at least c outputs come from A
        const bool pass = c <= hi && !less(src[pad16(b0 + k - c)], src[pad16(a0 + c - 1)]);
        const int t = __popcll(__ballot(pass));  // the passing lanes are a prefix
        lo += t * step;
        hi = hi < lo + step - 1 ? hi : lo + step - 1;
    }
    return lo;
}

// One LDS merge level of a full block, one wave per 64 PER consecutive
// outputs [o, o + 64 PER) of the merge of the pair of runs of length L that
// starts at s (L >= 64 PER).  The wave finds where its outputs start and end
// on both runs (wave_merge_path), loads its A slice ascending followed by its
// B slice descending -- a bitonic sequence -- lane-striped (element e in
// register e / 64 of lane e % 64, so consecutive lanes read consecutive LDS
// words), sorts it with the half-cleaners of a bitonic merge (distances of 64
// and more inside the lane, below 64 across lanes) and stores it striped.
template <int PER, typename W, typename Less>
__device__ __forceinline__ void wave_lds_merge(const W* src, W* dst, int s, int L, int o, int lane, Less less)
{
    constexpr int OUT = 64 * PER;
    const int a0 = s, b0 = s + L;
    const int k = o - s;
    const int i0 = wave_merge_path(src, a0, b0, L, k, lane, less);
    const int i1 = wave_merge_path(src, a0, b0, L, k + OUT, lane, less);
    const int na = i1 - i0;
    const int b_last = b0 + (k + OUT - i1) - 1;  // the B slice's last element
    W x[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int e = q * 64 + lane;
        x[q] = src[pad16(e < na ? a0 + i0 + e : b_last - (e - na))];
    }
#pragma unroll
    for (int d = PER / 2; d >= 1; d >>= 1) {  // distances 64 d, inside the lane
#pragma unroll
        for (int q = 0; q < PER; ++q)
            if ((q & d) == 0)
                order2(x[q], x[q + d], less);
    }
    half_clean_lanes<32>(x, lane, less);
#pragma unroll
    for (int q = 0; q < PER; ++q)
        dst[pad16(o + q * 64 + lane)] = x[q];
}

template <int KB, int VB>
__global__ __launch_bounds__((block_threads<KB, VB>())) void merge_block_sort_kernel(MergeBlockArgs a,
                                                                             OrderMap<typename KeyWord<KB>::U> om,
                                                                             int t_ins, int block_keys)
{
    using U = typename KeyWord<KB>::U;
    using V = typename ValWord<VB>::T;
    using R = BlockRec<KB, VB>;
    using W = typename R::W;
    constexpr int CAP = block_cap<KB, VB>();
    constexpr int THREADS = block_threads<KB, VB>();
    __shared__ W buf[2][padded16(CAP)];
    __shared__ V vpark[VB ? CAP : 1];

    const int64_t start = (int64_t)blockIdx.x * block_keys;
    const int64_t left = a.n - start;
    const int nb = left < block_keys ? (int)left : block_keys;
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);

    // Load the block.  Values are parked in LDS now, so that writing them
    // back over vals_in (in place) cannot race with reading them.  A thread's
    // loads are all issued before any of them is waited for: they carry no
    // branch, a position past the block reads its last key instead.
    constexpr int LOADS = CAP / THREADS;
    {
        U kr[LOADS];
        V vr[VB ? LOADS : 1];
        const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const int i0 = threadIdx.x + q * THREADS;
            const int i = i0 < nb ? i0 : nb - 1;
            kr[q] = keys_in[start + i];
            if constexpr (VB != 0)
                vr[q] = a.iota ? (V)(start + i) : vals_in[start + i];
        }
#pragma unroll
        for (int q = 0; q < LOADS; ++q) {
            const int i = threadIdx.x + q * THREADS;
            if (i < nb) {
                buf[0][pad16(i)] = R::make(om.to_order(kr[q]), (uint32_t)i);
                if constexpr (VB != 0)
                    vpark[i] = vr[q];
            }
        }
    }
    __syncthreads();

    constexpr int PER = kBlockPer;
    const auto less = [](const W& x, const W& y) { return R::less(x, y); };
    int first_lds_run = t_ins;  // run length of the first merge level done in LDS
    if (PER % t_ins == 0 && nb == CAP) {
        // A full block whose chunks tile each thread's PER records: the
        // thread sorts its records in registers with a bitonic sorting
        // network, which gives what sorting its chunks and merging them up to
        // runs of PER gives.  Records with values carry distinct positions,
        // and bare words that compare equal are identical, so the network's
        // order is the stable one.  The merge levels up to runs of one wave's
        // 64 PER records follow in registers too.
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
                        if ((q & size) == 0)
                            order2(x[q], x[pq], less);
                        else
                            order2(x[pq], x[q], less);
                    }
                }
            }
        }
        wave_merge_levels<PER, PER>(x, (int)(threadIdx.x & (kWave - 1)), less);
        first_lds_run = kWave * PER;
#pragma unroll
        for (int q = 0; q < PER; ++q)
            buf[1][pad16(c0 + q)] = x[q];
    } else {
        // Chunks of t_ins: place each record at (chunk start + number of
        // smaller records in its chunk).
        for (int i = threadIdx.x; i < nb; i += THREADS) {
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

    // Pairwise merges inside the block, run length doubling from t_ins (or
    // from the wave's run); on equal records the left run's goes first.
    // Thread t owns outputs [t*PER, (t+1)*PER) of every level.
    int cur = 1;
    if (first_lds_run == kWave * PER) {
        // the register path's block: full, runs of one wave's records; each
        // wave merges its share of every level (wave_lds_merge)
        const int lane = (int)(threadIdx.x & (kWave - 1));
        const int o = (int)(threadIdx.x / kWave) * kWave * PER;
        for (int L = first_lds_run; L < CAP; L *= 2) {
            wave_lds_merge<PER>(buf[cur], buf[cur ^ 1], (o / (2 * L)) * (2 * L), L, o, lane, less);
            __syncthreads();
            cur ^= 1;
        }
    }
    for (int L = first_lds_run; L < nb && first_lds_run != kWave * PER; L *= 2) {
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
    for (int i = threadIdx.x; i < nb; i += THREADS) {
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

    // the tile's A slice, then its B slice (element i of the tile is
    // a_base[i] or b_base[i]); a thread's loads are all issued before any of
    // them is waited for: they carry no branch, a position past the tile
    // reads the tile's last element instead (cnt >= 1 here)
    const U* keys_in = reinterpret_cast<const U*>(a.keys_in);
    const V* vals_in = reinterpret_cast<const V*>(a.vals_in);
    const int64_t a_base = s + a0, b_base = s + na + b0 - ca;
    {
        U kr[PER];
        V vr[VB ? PER : 1];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int i0 = threadIdx.x + q * kRoundThreads;
            const int i = i0 < cnt ? i0 : cnt - 1;
            const int64_t src = (i < ca ? a_base : b_base) + i;
            kr[q] = keys_in[src];
            if constexpr (VB != 0)
                vr[q] = vals_in[src];
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
    hipLaunchKernelGGL((merge_block_sort_kernel<KB, VB>), dim3((unsigned)mp.blocks), dim3(block_threads<KB, VB>()), 0, s, a,
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
