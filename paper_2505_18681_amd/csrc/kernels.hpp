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

// Exclusive prefix sums of each pass's 2^bits histogram row.
hipError_t launch_radix_scan(const uint64_t* hist, uint64_t* bases, int bits, int passes, hipStream_t s);

struct RadixPassArgs {
    const void* keys_in;
    void* keys_out;
    const void* vals_in;  // unused when val_bytes == 0 or iota
    void* vals_out;
    int64_t n;
    uint32_t shift;          // bit offset of this pass's digit in the order word
    const uint64_t* bases;   // 2^bits first output slots of each digit
    void* status;            // tiles * 2^bits look-back words (zeroed)
    uint32_t* tile_counter;  // zeroed
    uint32_t* error_word;    // device error word in the scratch header
    uint32_t* host_error;    // host-visible word also set on a device-side error (may be null)
    uint32_t flags;          // RADIX_FLAG_*
    uint32_t spin_limit;
    uint32_t tiles;          // workgroups launched (= tiles of the pass)
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
hipError_t launch_radix_pass(const KeyDesc& kd, int val_bytes, int bits, RadixShape shape, int status_bytes,
                             const RadixPassArgs& a, uint32_t tiles, hipStream_t s);

// ---------------------------------------------------------------- misc -----

// Zero `bytes` bytes at p (16-byte stores when p and bytes allow).
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);

// Copy `bytes` bytes device to device (a runtime copy on stream s).
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t s);

}  // namespace evosort
