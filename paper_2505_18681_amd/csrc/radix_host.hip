// Launchers of the radix histogram and scan kernels, the utility kernels, and
// the dispatch of the pass kernel over (key bytes, value bytes).
#include "radix_impl.hpp"
#include "radix_shapes.hpp"

namespace evosort {

hipError_t radix_pass_dispatch_k4_v0(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);
hipError_t radix_pass_dispatch_k4_v4(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);
hipError_t radix_pass_dispatch_k4_v8(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);
hipError_t radix_pass_dispatch_k8_v0(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);
hipError_t radix_pass_dispatch_k8_v4(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);
hipError_t radix_pass_dispatch_k8_v8(int, RadixShape, int, const KeyDesc&, const RadixPassArgs&, uint32_t,
                                     hipStream_t, bool*);

hipError_t seg_pass_dispatch_k4_v0(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);
hipError_t seg_pass_dispatch_k4_v4(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);
hipError_t seg_pass_dispatch_k4_v8(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);
hipError_t seg_pass_dispatch_k8_v0(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);
hipError_t seg_pass_dispatch_k8_v4(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);
hipError_t seg_pass_dispatch_k8_v8(RadixShape, const KeyDesc&, const SegPassArgs&, uint32_t, hipStream_t, bool*);

// Compute units of the MI355X (gfx950) the size-dependent grids and tiles are
// chosen for.
constexpr int64_t kComputeUnits = 256;

namespace {
constexpr int kHistThreads = 256;

int histogram_grid(int64_t n)
{
    // Enough workgroups to fill 256 CUs several times over; each thread then
    // walks the keys with a grid stride.  Up to 2^23 keys at most one per CU:
    // every workgroup flushes its counts into the same few global words with
    // atomics, and beyond one workgroup per CU those flushes cost more than
    // the reads they spread (4-byte keys 2 to 9 % faster from 1.1e6 to 4.6e6
    // keys; 8-byte keys within 1 %).
    int64_t want = (n + 16 * kHistThreads - 1) / (16 * kHistThreads);
    if (want < 1)
        want = 1;
    if (want > 4096)
        want = 4096;
    if (n <= (int64_t)1 << 23 && want > kComputeUnits)
        want = kComputeUnits;
    return (int)want;
}
}  // namespace

hipError_t launch_radix_histogram(const KeyDesc& kd, const void* keys, int64_t n, int bits, int passes,
                                  uint64_t* hist, hipStream_t s)
{
    // LDS budget of one launch: 64 KB of 32-bit counters.  Group the passes so
    // that each group has at least one private copy; add copies (at most one
    // per wave) while they fit.
    const size_t per_pass = ((size_t)1 << bits) * 4;
    if (bits == 8 && (passes == 4 || passes == 8)) {
        // every pass in one launch, one set of counters per workgroup (as in
        // launch_radix_histogram_tiles)
        const int grid = histogram_grid(n);
        const int copies = 1;
        const size_t lds = (size_t)copies * passes * per_pass;
        auto* h = reinterpret_cast<unsigned long long*>(hist);
        if (kd.bytes == 4 && passes == 4) {
            OrderMap<uint32_t> om{(uint32_t)kd.flip, (uint32_t)kd.neg, (uint32_t)kd.desc};
            hipLaunchKernelGGL((radix_histogram8_kernel<4, kHistThreads, 4>), dim3(grid), dim3(kHistThreads), lds,
                               s, reinterpret_cast<const uint32_t*>(keys), n, om, copies, h);
            return hipGetLastError();
        }
        if (kd.bytes == 8 && passes == 8) {
            OrderMap<uint64_t> om{kd.flip, kd.neg, kd.desc};
            hipLaunchKernelGGL((radix_histogram8_kernel<8, kHistThreads, 8>), dim3(grid), dim3(kHistThreads), lds,
                               s, reinterpret_cast<const uint64_t*>(keys), n, om, copies, h);
            return hipGetLastError();
        }
    }
    const int group = (int)((64 * 1024) / per_pass) < passes ? (int)((64 * 1024) / per_pass) : passes;
    const int grid = histogram_grid(n);
    auto* h = reinterpret_cast<unsigned long long*>(hist);
    for (int p0 = 0; p0 < passes; p0 += group) {
        const int np = passes - p0 < group ? passes - p0 : group;
        int copies = (int)((64 * 1024) / (per_pass * np));
        if (copies > kHistThreads / kWave)
            copies = kHistThreads / kWave;
        if (copies < 1)
            copies = 1;
        const size_t lds = (size_t)copies * np * per_pass;
        if (kd.bytes == 4) {
            OrderMap<uint32_t> om{(uint32_t)kd.flip, (uint32_t)kd.neg, (uint32_t)kd.desc};
            hipLaunchKernelGGL((radix_histogram_kernel<4, kHistThreads>), dim3(grid), dim3(kHistThreads), lds, s,
                               reinterpret_cast<const uint32_t*>(keys), n, om, bits, p0, np, copies, h);
        } else {
            OrderMap<uint64_t> om{kd.flip, kd.neg, kd.desc};
            hipLaunchKernelGGL((radix_histogram_kernel<8, kHistThreads>), dim3(grid), dim3(kHistThreads), lds, s,
                               reinterpret_cast<const uint64_t*>(keys), n, om, bits, p0, np, copies, h);
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess)
            return e;
    }
    return hipSuccess;
}

hipError_t launch_radix_histogram_tiles(const KeyDesc& kd, const void* keys, int64_t n, int passes,
                                        uint64_t* hist, void* counts, int status_bytes, uint32_t tile_keys,
                                        uint32_t tiles, hipStream_t s)
{
    if (tiles == 0)
        return hipSuccess;
    // One set of counters per workgroup: LDS atomics of different waves on
    // one counter are separate instructions and do not conflict, and the
    // smaller footprint lets more workgroups share a CU (one copy per wave:
    // 1e9 int64 keys 2.32 ms, one per workgroup 2.16 ms; int32 keys equal).
    const int copies = 1;
    const size_t lds = ((size_t)copies * passes + 1) * 256 * 4;
    // Workgroups stride over the tiles, about three tiles each, between 2048
    // and 16384 workgroups: every workgroup flushes its counts with global
    // atomics, so fewer of them flush less, while 16384 keep the largest
    // arrays' reads in flight (int32 keys: 1e9 1.06 ms with 16384 against
    // 1.10 and 1.07 with 4096 and 8192; 1e8 0.158 ms with 2048 against 0.181
    // with one workgroup per tile).  The kernel is bound by the throughput
    // of its LDS atomics: 4 per 4-byte key, one per digit position.
    const uint32_t third = tiles / 3;
    const uint32_t want = third < 2048 ? 2048 : (third > 16384 ? 16384 : third);
    const uint32_t grid = tiles < want ? tiles : want;
    auto* h = reinterpret_cast<unsigned long long*>(hist);
#define EVOSORT_HT(KB, P, ST, U)                                                                                 \
    do {                                                                                                       \
        OrderMap<U> om{(U)kd.flip, (U)kd.neg, (U)kd.desc};                                                                 \
        hipLaunchKernelGGL((radix_histogram8_tiles_kernel<KB, kHistThreads, P, ST>), dim3(grid),                \
                           dim3(kHistThreads), lds, s, reinterpret_cast<const U*>(keys), n, om, copies, h,      \
                           reinterpret_cast<ST*>(counts), tile_keys, tiles);                                   \
        return hipGetLastError();                                                                              \
    } while (0)
    if (kd.bytes == 4 && passes == 4) {
        if (status_bytes == 4)
            EVOSORT_HT(4, 4, uint32_t, uint32_t);
        EVOSORT_HT(4, 4, uint64_t, uint32_t);
    }
    if (kd.bytes == 8 && passes == 8) {
        if (status_bytes == 4)
            EVOSORT_HT(8, 8, uint32_t, uint64_t);
        EVOSORT_HT(8, 8, uint64_t, uint64_t);
    }
#undef EVOSORT_HT
    return hipErrorInvalidValue;
}

hipError_t launch_tile_prefix(void* counts, int status_bytes, uint32_t tiles, uint64_t* block_sums, hipStream_t s)
{
    if (tiles == 0)
        return hipSuccess;
    const uint32_t blocks = (tiles + kTilePrefixBlock - 1) / kTilePrefixBlock;
    if (status_bytes == 4)
        hipLaunchKernelGGL(tile_block_sum_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint32_t*>(counts), tiles, block_sums);
    else
        hipLaunchKernelGGL(tile_block_sum_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<const uint64_t*>(counts), tiles, block_sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(tile_block_scan_kernel<256>, dim3(256), dim3(256), 0, s, block_sums, blocks);
    e = hipGetLastError();
    if (e != hipSuccess)
        return e;
    if (status_bytes == 4)
        hipLaunchKernelGGL(tile_prefix_kernel<uint32_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<uint32_t*>(counts), tiles, block_sums);
    else
        hipLaunchKernelGGL(tile_prefix_kernel<uint64_t>, dim3(blocks), dim3(256), 0, s,
                           reinterpret_cast<uint64_t*>(counts), tiles, block_sums);
    return hipGetLastError();
}

hipError_t launch_radix_scan(const uint64_t* hist, uint64_t* bases, int bits, int passes, uint32_t* live,
                             uint32_t* done, unsigned long long* tickets, hipStream_t s)
{
    hipLaunchKernelGGL((radix_scan_kernel<256>), dim3(passes), dim3(256), 0, s, hist, bases, 1 << bits, live, done,
                       tickets);
    return hipGetLastError();
}

RadixShape radix_default_shape(int key_bytes, int val_bytes, int bits)
{
    const RadixShape def = radix_default_shape_c(key_bytes, val_bytes);
    if (radix_lds_bytes(key_bytes, val_bytes, bits, def.threads, def.items) <= kLdsLimit)
        return def;
    return kRadixFallbackShape;
}

// Arrays of up to a few million keys have too few default tiles to fill the
// 256 CUs (1e5 int32 keys: 6 tiles of 18432), and a pass is launch- and
// latency-bound there.  Smaller tiles at 8-bit digits, measured on int32 keys
// (ms per sort, default tile against this one): 3e4 0.149 / 0.112, 1e5 0.153 /
// 0.116, 3e5 0.163 / 0.136 with 512 x 8; 1e6 0.182 / 0.155 with 512 x 16; at
// 3e6 the default is within 2 %.  1e5 int64 keys: 0.216 / 0.189; 1e5 int32
// keys with 8-byte values: 0.148 / 0.123.
RadixShape radix_default_shape_for(int key_bytes, int val_bytes, int bits, int64_t n)
{
    if (bits == 8 && n <= (int64_t)1 << 19)
        return RadixShape{512, 8};
    // From 2^19 to 2^21 keys 768 x 12 for every key and value width: it beat
    // 512 x 16 at every size swept there, keys only and pairs (2 to 3.5 % on
    // average, up to 9 %)
    if (bits == 8 && n <= (int64_t)1 << 21)
        return RadixShape{768, 12};
    // Pairs with an 8-byte word among key and value, between 2^21 and 2^26
    // keys: 768 x 16 (one 8-byte word) and 768 x 12 (8-byte keys and values)
    // beat the large-array tiles 512 x 24 and 512 x 16 at every size swept
    // there (5 to 6 % on average); the large-array tiles were chosen at 1e9.
    if (bits == 8 && n > (int64_t)1 << 21 && n <= (int64_t)1 << 26 && (key_bytes == 8 || val_bytes == 8) &&
        val_bytes != 0)
        return key_bytes + val_bytes == 12 ? RadixShape{768, 16} : RadixShape{768, 12};
    if (bits == 8 && key_bytes == 4 && val_bytes != 8 && n <= (int64_t)1 << 26) {
        // Up to some tens of tiles per CU, a pass lasts about as long as its
        // busiest CU takes to stream its tiles: ceil(tiles / CUs) tiles of T
        // keys.  Take the shape that puts the fewest keys on the busiest CU
        // (the larger tile on ties).  At 2.5e6 to 8e6 keys this picked the
        // fastest of five shapes at 7 of 8 sizes swept (4.6 % faster than
        // 768 x 24 on average); above 2^23 keys the 1024 x 20 and smaller
        // tiles lose more per key than the rounding gains, and the choice is
        // between 768 x 24 and 1024 x 16 only (1 to 4 % where it switches).
        // Pairs with 4-byte values (and argsort with 32-bit indices) take the
        // same rule over the shapes compiled for them (3.3 % faster on
        // average over 24 sizes from 2.2e6 to 6.6e7 keys, at most 0.4 %
        // slower).
        constexpr RadixShape kShapes[] = {{768, 24}, {1024, 16}, {1024, 20}, {768, 20}, {768, 16}};
        const int count = n <= (int64_t)1 << 23 ? 5 : 2;
        RadixShape best = kShapes[0];
        int64_t best_keys = -1, best_tile = 0;
        for (int k = 0; k < count; ++k) {
            const RadixShape& c = kShapes[k];
            if (!radix_pass_available(key_bytes, val_bytes, bits, c, 4))  // same set at either word width
                continue;
            const int64_t tile = (int64_t)c.threads * c.items;
            const int64_t per_cu = ((n + tile - 1) / tile + kComputeUnits - 1) / kComputeUnits * tile;
            if (best_keys < 0 || per_cu < best_keys || (per_cu == best_keys && tile > best_tile)) {
                best = c;
                best_keys = per_cu;
                best_tile = tile;
            }
        }
        return best;
    }
    return radix_default_shape(key_bytes, val_bytes, bits);
}

bool radix_pass_available(int key_bytes, int val_bytes, int bits, RadixShape sh, int status_bytes)
{
    if (key_bytes != 4 && key_bytes != 8)
        return false;
    if (val_bytes != 0 && val_bytes != 4 && val_bytes != 8)
        return false;
    if (bits < 4 || bits > 12 || (status_bytes != 4 && status_bytes != 8))
        return false;
    if (radix_lds_bytes(key_bytes, val_bytes, bits, sh.threads, sh.items) > kLdsLimit)
        return false;
    const RadixShape def = radix_default_shape_c(key_bytes, val_bytes);
    if (sh.threads == def.threads && sh.items == def.items)
        return true;
    if (sh.threads == kRadixFallbackShape.threads && sh.items == kRadixFallbackShape.items)
        return true;
    if (bits != 8)
        return false;
#define EVOSORT_MATCH_SHAPE(T, I)                 \
    if (sh.threads == (T) && sh.items == (I))     \
        return true;
    EVOSORT_RADIX_ALT_SHAPES(EVOSORT_MATCH_SHAPE)
#undef EVOSORT_MATCH_SHAPE
    return false;
}

hipError_t launch_radix_pass(const KeyDesc& kd, int val_bytes, int bits, RadixShape shape, int status_bytes,
                             const RadixPassArgs& a, uint32_t tiles, hipStream_t s)
{
    bool found = false;
    hipError_t e = hipErrorInvalidValue;
    if (kd.bytes == 4) {
        if (val_bytes == 0)
            e = radix_pass_dispatch_k4_v0(bits, shape, status_bytes, kd, a, tiles, s, &found);
        else if (val_bytes == 4)
            e = radix_pass_dispatch_k4_v4(bits, shape, status_bytes, kd, a, tiles, s, &found);
        else
            e = radix_pass_dispatch_k4_v8(bits, shape, status_bytes, kd, a, tiles, s, &found);
    } else {
        if (val_bytes == 0)
            e = radix_pass_dispatch_k8_v0(bits, shape, status_bytes, kd, a, tiles, s, &found);
        else if (val_bytes == 4)
            e = radix_pass_dispatch_k8_v4(bits, shape, status_bytes, kd, a, tiles, s, &found);
        else
            e = radix_pass_dispatch_k8_v8(bits, shape, status_bytes, kd, a, tiles, s, &found);
    }
    if (!found)
        return hipErrorInvalidValue;
    return e;
}

// Tile shapes of the long segments of a batch (around 1e5 to 4e6 keys each),
// measured on the 100k-array batch: keys-only 4-byte keys take the
// single-array default, 768 x 24 (15.85 ms against 16.25 ms with 512 x 24 and
// 16.55 ms with 1024 x 16); pairs keep 8-wave tiles.
RadixShape seg_default_shape(int key_bytes, int val_bytes)
{
    if (key_bytes == 4)
        return val_bytes == 0 ? RadixShape{768, 24} : (val_bytes == 4 ? RadixShape{512, 16} : RadixShape{512, 24});
    return val_bytes == 4 ? RadixShape{512, 24} : RadixShape{512, 16};
}

bool seg_pass_available(int key_bytes, int val_bytes, RadixShape sh)
{
    if ((key_bytes != 4 && key_bytes != 8) || (val_bytes != 0 && val_bytes != 4 && val_bytes != 8))
        return false;
    if (radix_lds_bytes(key_bytes, val_bytes, kSegBits, sh.threads, sh.items) > kLdsLimit)
        return false;
#define EVOSORT_MATCH_SEG_SHAPE(T, I)             \
    if (sh.threads == (T) && sh.items == (I))     \
        return true;
    EVOSORT_SEG_SHAPES(EVOSORT_MATCH_SEG_SHAPE)
#undef EVOSORT_MATCH_SEG_SHAPE
    return false;
}

hipError_t launch_seg_radix_pass(const KeyDesc& kd, int val_bytes, RadixShape shape, const SegPassArgs& a,
                                 uint32_t grid, hipStream_t s)
{
    bool found = false;
    hipError_t e = hipErrorInvalidValue;
    if (kd.bytes == 4) {
        if (val_bytes == 0)
            e = seg_pass_dispatch_k4_v0(shape, kd, a, grid, s, &found);
        else if (val_bytes == 4)
            e = seg_pass_dispatch_k4_v4(shape, kd, a, grid, s, &found);
        else
            e = seg_pass_dispatch_k4_v8(shape, kd, a, grid, s, &found);
    } else {
        if (val_bytes == 0)
            e = seg_pass_dispatch_k8_v0(shape, kd, a, grid, s, &found);
        else if (val_bytes == 4)
            e = seg_pass_dispatch_k8_v4(shape, kd, a, grid, s, &found);
        else
            e = seg_pass_dispatch_k8_v8(shape, kd, a, grid, s, &found);
    }
    if (!found)
        return hipErrorInvalidValue;
    return e;
}

// ------------------------------------------------------------------ misc ---

__global__ __launch_bounds__(256) void fill_zero_kernel(uint4* p, size_t n16)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0, 0, 0, 0);
}

__global__ __launch_bounds__(256) void fill_zero_bytes_kernel(unsigned char* p, size_t bytes)
{
    const size_t stride = (size_t)gridDim.x * 256;
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < bytes; i += stride)
        p[i] = 0;
}

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    if ((bytes & 15) || (reinterpret_cast<uintptr_t>(p) & 15)) {
        size_t grid = (bytes + 255) / 256;
        if (grid > 8192)
            grid = 8192;
        hipLaunchKernelGGL(fill_zero_bytes_kernel, dim3((unsigned)grid), dim3(256), 0, s,
                           reinterpret_cast<unsigned char*>(p), bytes);
        return hipGetLastError();
    }
    const size_t n16 = bytes / 16;
    size_t grid = (n16 + 255) / 256;
    if (grid > 8192)
        grid = 8192;
    if (grid < 1)
        grid = 1;
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)grid), dim3(256), 0, s, reinterpret_cast<uint4*>(p), n16);
    return hipGetLastError();
}

// ---------------------------------------------------------------- streams --
// Streaming copy and read: every byte moved once, 16-byte accesses with eight
// of them in flight per thread, a grid-stride loop over the range.  The copy
// is the library's device-to-device copy; both are also the practical
// ceilings the radix pass (read and write once) and the histogram (read
// once) are measured against.
constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 8;  // 16-byte words in flight per thread in the streaming kernels

uint32_t stream_grid(size_t bytes)
{
    const size_t per_group = (size_t)kStreamThreads * kStreamUnroll * 16;
    size_t g = (bytes + per_group - 1) / per_group;
    if (g < 1)
        g = 1;
    if (g > 16384)
        g = 16384;
    return (uint32_t)g;
}

// bytes is a multiple of 4 (keys, values and indices are 4 or 8 bytes).
__device__ __forceinline__ void copy_range(unsigned char* __restrict__ dst, const unsigned char* __restrict__ src,
                                           size_t bytes, size_t tid, size_t nthreads)
{
    size_t done = 0;
    if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15) == 0) {
        const size_t n16 = bytes / 16;
        uint4* d = reinterpret_cast<uint4*>(dst);
        const uint4* s = reinterpret_cast<const uint4*>(src);
        size_t i = tid;
        // eight 16-byte words in flight per thread
        for (; i + 7 * nthreads < n16; i += 8 * nthreads) {
            const uint4 w0 = s[i], w1 = s[i + nthreads], w2 = s[i + 2 * nthreads], w3 = s[i + 3 * nthreads];
            const uint4 w4 = s[i + 4 * nthreads], w5 = s[i + 5 * nthreads], w6 = s[i + 6 * nthreads],
                        w7 = s[i + 7 * nthreads];
            // every load is issued before the first store: the scheduler
            // would otherwise pair each load with its store and wait on each
            __builtin_amdgcn_sched_barrier(0);
            d[i] = w0;
            d[i + nthreads] = w1;
            d[i + 2 * nthreads] = w2;
            d[i + 3 * nthreads] = w3;
            d[i + 4 * nthreads] = w4;
            d[i + 5 * nthreads] = w5;
            d[i + 6 * nthreads] = w6;
            d[i + 7 * nthreads] = w7;
        }
        for (; i < n16; i += nthreads)
            d[i] = s[i];
        done = n16 * 16;
    }
    uint32_t* d4 = reinterpret_cast<uint32_t*>(dst + done);
    const uint32_t* s4 = reinterpret_cast<const uint32_t*>(src + done);
    for (size_t i = tid; i < (bytes - done) / 4; i += nthreads)
        d4[i] = s4[i];
}

__global__ __launch_bounds__(kStreamThreads) void stream_copy_kernel(unsigned char* dst, const unsigned char* src,
                                                                     size_t bytes)
{
    copy_range(dst, src, bytes, (size_t)blockIdx.x * kStreamThreads + threadIdx.x,
               (size_t)gridDim.x * kStreamThreads);
}

// Reads every 16-byte word once (bytes: a multiple of 16, 16-byte aligned)
// and folds it into one word per thread; a thread stores its word only when it
// equals a value a real input practically never produces, so the loads cannot
// be dropped and the kernel writes (almost) nothing.
__global__ __launch_bounds__(kStreamThreads) void stream_read_kernel(const uint4* __restrict__ src, size_t n16,
                                                                     unsigned long long* sink)
{
    const size_t nthreads = (size_t)gridDim.x * kStreamThreads;
    size_t i = (size_t)blockIdx.x * kStreamThreads + threadIdx.x;
    uint32_t acc = 0;
    for (; i + (kStreamUnroll - 1) * nthreads < n16; i += kStreamUnroll * nthreads) {
        uint4 w[kStreamUnroll];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
            w[u] = src[i + u * nthreads];
#pragma unroll
        for (int u = 0; u < kStreamUnroll; ++u)
            acc = (acc * 31u) ^ w[u].x ^ w[u].y ^ w[u].z ^ w[u].w;
    }
    for (; i < n16; i += nthreads) {
        const uint4 w = src[i];
        acc = (acc * 31u) ^ w.x ^ w.y ^ w.z ^ w.w;
    }
    if (acc == 0x9E3779B9u)
        sink[0] = acc;
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    if (bytes == 0 || dst == src)
        return hipSuccess;
    if (bytes & 3)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_copy_kernel, dim3(stream_grid(bytes)), dim3(kStreamThreads), 0, s,
                       reinterpret_cast<unsigned char*>(dst), reinterpret_cast<const unsigned char*>(src), bytes);
    return hipGetLastError();
}

// After the passes of a routed sort (see RadixRoute): with no live pass, the
// input goes to the output unchanged (argsort: the identity permutation);
// with an odd number of live passes sorted in place, the last pass's
// temporary buffer goes to the output; otherwise every workgroup leaves.
__global__ __launch_bounds__(kStreamThreads) void radix_finish_kernel(RadixRoute r, int64_t n, int kb, int vb)
{
    const uint32_t m = (uint32_t)__builtin_popcount(*r.live);
    const size_t tid = (size_t)blockIdx.x * kStreamThreads + threadIdx.x;
    const size_t nth = (size_t)gridDim.x * kStreamThreads;
    const bool argsort = (r.flags & ROUTE_ARGSORT) != 0;
    if (m == 0) {
        if (argsort) {
            if (vb == 4) {
                for (size_t i = tid; i < (size_t)n; i += nth)
                    reinterpret_cast<uint32_t*>(r.vals_out)[i] = (uint32_t)i;
            } else {
                for (size_t i = tid; i < (size_t)n; i += nth)
                    reinterpret_cast<uint64_t*>(r.vals_out)[i] = (uint64_t)i;
            }
            return;
        }
        if (r.keys_out != r.keys_in)
            copy_range(reinterpret_cast<unsigned char*>(r.keys_out), reinterpret_cast<const unsigned char*>(r.keys_in),
                       (size_t)n * kb, tid, nth);
        if (vb && r.vals_out != r.vals_in)
            copy_range(reinterpret_cast<unsigned char*>(r.vals_out), reinterpret_cast<const unsigned char*>(r.vals_in),
                       (size_t)n * vb, tid, nth);
        return;
    }
    if (!argsort && (r.flags & ROUTE_COPY_IF_ODD) && (m & 1)) {
        copy_range(reinterpret_cast<unsigned char*>(r.keys_out), reinterpret_cast<const unsigned char*>(r.keys_tmp),
                   (size_t)n * kb, tid, nth);
        if (vb)
            copy_range(reinterpret_cast<unsigned char*>(r.vals_out), reinterpret_cast<const unsigned char*>(r.vals_tmp),
                       (size_t)n * vb, tid, nth);
    }
}

hipError_t launch_radix_finish(const RadixRoute& r, int64_t n, int key_bytes, int val_bytes, hipStream_t s)
{
    if (n <= 0 || !r.live)
        return hipSuccess;
    hipLaunchKernelGGL(radix_finish_kernel, dim3(stream_grid((size_t)n * (key_bytes > val_bytes ? key_bytes : val_bytes))),
                       dim3(kStreamThreads), 0, s, r, n, key_bytes, val_bytes);
    return hipGetLastError();
}

hipError_t launch_stream_read(const void* src, size_t bytes, uint64_t* sink, hipStream_t s)
{
    if (bytes == 0)
        return hipSuccess;
    if ((bytes & 15) || (reinterpret_cast<uintptr_t>(src) & 15))
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(stream_read_kernel, dim3(stream_grid(bytes)), dim3(kStreamThreads), 0, s,
                       reinterpret_cast<const uint4*>(src), bytes / 16,
                       reinterpret_cast<unsigned long long*>(sink));
    return hipGetLastError();
}

}  // namespace evosort
