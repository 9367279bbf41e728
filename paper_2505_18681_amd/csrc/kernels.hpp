// Launchers of the library's kernels.  Host code (the C ABI) calls only these;
// each returns the hipError_t of its launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace evosort {

// Word-level description of a key type (see OrderMap in common.hpp).
struct KeyDesc {
    int bytes;      // 4 or 8
    uint64_t flip;  // XOR applied to every key word
    uint64_t neg;   // extra XOR for keys whose sign bit is set (floats: all ones)
    uint64_t desc;  // all ones for descending order (the order word complemented), else 0
};

// ---------------------------------------------------------------- radix ----

// One read of the keys: histograms of every digit position, added into
// hist[passes << bits] (uint64, zeroed by the caller).  When all passes do not
// fit in LDS at once the passes are split over several launches.
hipError_t launch_radix_histogram(const KeyDesc& kd, const void* keys, int64_t n, int bits, int passes,
                                  uint64_t* hist, hipStream_t s);

// The all-pass histogram of 8-bit digits (passes 4 or 8, zeroed hist) that
// also writes, for every tile of tile_keys keys, the tile's counts of the
// pass-0 digits: counts[tile * 256 + digit], words of status_bytes (4 or 8).
hipError_t launch_radix_histogram_tiles(const KeyDesc& kd, const void* keys, int64_t n, int passes,
                                        uint64_t* hist, void* counts, int status_bytes, uint32_t tile_keys,
                                        uint32_t tiles, hipStream_t s);

// Turns the per-tile counts of launch_radix_histogram_tiles, in place, into
// each tile's exclusive prefix per digit (the sum over all earlier tiles).
// block_sums: scratch of ceil(tiles / 64) * 256 uint64.
hipError_t launch_tile_prefix(void* counts, int status_bytes, uint32_t tiles, uint64_t* block_sums, hipStream_t s);
constexpr uint32_t kTilePrefixBlock = 64;  // tiles per workgroup of the prefix kernels

// Exclusive prefix sums of each pass's 2^bits histogram row.  With `live`
// (one word, zero before the launch) it also sets bit p when pass p's digit
// takes more than one value over the keys; a pass whose digit is the same for
// every key would leave the order unchanged.
// `done` (one zeroed word) and `tickets` (passes 64-bit ticket counters,
// zeroed) go with `live`: the last scan workgroup writes each pass's route
// code (route_code below) into the upper half of that pass's ticket counter.
hipError_t launch_radix_scan(const uint64_t* hist, uint64_t* bases, int bits, int passes, uint32_t* live,
                             uint32_t* done, unsigned long long* tickets, hipStream_t s);

// Route code of a pass in the upper half of its ticket counter: routed, live,
// its index j among the live passes and their number m.
constexpr uint32_t kRouteOn = 1u;
constexpr uint32_t kRouteLive = 2u;
__host__ __device__ constexpr uint32_t route_code(uint32_t live, uint32_t j, uint32_t m)
{
    return kRouteOn | (live ? kRouteLive : 0u) | (j << 8) | (m << 16);
}
__host__ __device__ constexpr uint32_t route_j(uint32_t code) { return (code >> 8) & 0xffu; }
__host__ __device__ constexpr uint32_t route_m(uint32_t code) { return (code >> 16) & 0xffu; }

// Buffers of a whole radix sort, from which each pass picks its input and
// output on the device once the live passes are known (the scan's `live`
// word): the launch sequence stays the same whatever digits are constant.
// Live pass j (0-based among the m live passes) reads what live pass j - 1
// wrote (the input for j = 0) and writes
//   keys-only / pairs:  the output when m - 1 - j is even, else the
//                       temporary buffer; with ROUTE_COPY_IF_ODD (sorting in
//                       place) and m odd, the temporary buffer when j is even
//                       and the output when j is odd, and the finishing launch
//                       copies the temporary buffer to the output;
//   argsort:            keys to keys_tmp (j even) or keys_tmp2 (j odd), never
//                       the last live pass; indices as pairs' values, the
//                       first live pass taking the input positions.
// With no live pass the finishing launch copies the input to the output
// (argsort: writes the identity permutation).
struct RadixRoute {
    const uint32_t* live;  // the scan's live-pass word (read by the finishing launch); null: no routing
    uint32_t pass, passes;
    uint32_t flags;        // ROUTE_*
    const void* keys_in;
    void* keys_out;
    void* keys_tmp;
    void* keys_tmp2;       // argsort only
    const void* vals_in;   // pairs only
    void* vals_out;        // values or indices
    void* vals_tmp;
};
constexpr uint32_t ROUTE_ARGSORT = 1u;
constexpr uint32_t ROUTE_COPY_IF_ODD = 2u;

struct RadixPassArgs {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;  // unused when val_bytes == 0 or iota
    void* vals_out;
    int64_t n;
    uint32_t shift;          // bit offset of this pass's digit in the order word
    const uint64_t* bases;   // 2^bits first output slots of each digit
    void* status;            // tiles * 2^bits look-back words (zeroed)
    uint32_t* tile_counter;  // zeroed (segmented pass)
    unsigned long long* ticket;  // radix pass: tile in the lower half, route code in the upper (zeroed: none)
    uint32_t* error_word;    // device error word in the scratch header
    uint32_t* host_error;    // host-visible word also set on a device-side error (may be null)
    uint32_t flags;          // RADIX_FLAG_*
    uint32_t spin_limit;
    uint32_t tiles;          // workgroups launched (= tiles of the pass)
    RadixRoute route;        // used when the ticket carries a route code
};
constexpr uint32_t RADIX_FLAG_IOTA = 1u;          // values are the input positions (argsort, first pass)
constexpr uint32_t RADIX_FLAG_SKIP_KEYS = 2u;     // do not write keys (argsort, last pass)
constexpr uint32_t RADIX_FLAG_WITHHOLD_T0 = 4u;   // debug: tile 0 never publishes
constexpr uint32_t RADIX_FLAG_PREFIX = 8u;        // status holds each tile's exclusive digit prefixes, computed
                                                  // before the pass: no publication, no look-back

struct RadixShape {
    int threads;
    int items;
};

// Default tile shape for (key bytes, value bytes, digit bits): the preferred
// shape where it fits in LDS, else the fallback shape.
RadixShape radix_default_shape(int key_bytes, int val_bytes, int bits);
// The default shape for an array of n keys: smaller tiles for short arrays.
RadixShape radix_default_shape_for(int key_bytes, int val_bytes, int bits, int64_t n);
// Whether a single-sweep pass kernel exists for these parameters.
bool radix_pass_available(int key_bytes, int val_bytes, int bits, RadixShape shape, int status_bytes);
// The launch after the passes of a routed sort: the copy (or identity
// permutation) that the live passes leave to do, if any; n keys of key_bytes,
// values or indices of val_bytes.
hipError_t launch_radix_finish(const RadixRoute& r, int64_t n, int key_bytes, int val_bytes, hipStream_t s);
hipError_t launch_radix_pass(const KeyDesc& kd, int val_bytes, int bits, RadixShape shape, int status_bytes,
                             const RadixPassArgs& a, uint32_t tiles, hipStream_t s);

// ---------------------------------------------------------------- misc -----

// Zero `bytes` bytes at p (16-byte stores when p and bytes allow).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// Copy `bytes` bytes (a multiple of 4) device to device with the library's
// streaming copy kernel.
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);
// Read `bytes` bytes (a multiple of 16, 16-byte aligned) once, writing
// (almost) nothing: the ceiling of a read-only kernel.  sink: one device word.
hipError_t launch_stream_read(const void* src, size_t bytes, uint64_t* sink, hipStream_t s);

}  // namespace evosort
