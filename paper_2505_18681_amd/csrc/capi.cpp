// C ABI of the sort library: argument checks, the adaptive partition sort
// dispatch (Sec. 4.3, Algorithm 6), scratch layout, and the launch sequences
// of the radix, mergesort and one-workgroup routines.
#include <hip/hip_runtime.h>
#include <string.h>

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "capi_internal.hpp"
#include "evosort.h"
#include "kernels.hpp"
#include "merge.hpp"
#include "radix_shapes.hpp"
#include "segmented.hpp"
#include "small_sort.hpp"
#include "tuned_table.hpp"

using namespace evosort;

namespace {

thread_local int t_last_hip = 0;
// Set while the allocation-free sort runs: its launches are never bracketed
// by profiling events (creating an event may allocate).
thread_local bool t_no_events = false;

// ------------------------------------------------------ host error words --
// One host-visible word per device, in pinned host memory that the device
// maps coherently.  The kernels of a public call store an error bit there on
// a device-side failure (a look-back wait out of spins, bad segment offsets),
// besides the error word in the call's scratch.  The host reads it without
// synchronizing: the next public call on that device finds it nonzero,
// returns the error instead of running, and clears it.
struct HostErrorWords {
    std::mutex mu;
    std::map<int, uint32_t*> host;    // host address, per device
    std::map<int, uint32_t*> device;  // the same memory as kernels address it
};
HostErrorWords& host_error_words()
{
    static HostErrorWords* w = new HostErrorWords();  // never destroyed: outlives static teardown order
    return *w;
}

int current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return -1;
    }
    return dev;
}

// Kernel address of the current device's word, allocated on first use.  Not
// allocated while `s` is being captured into a graph (allocation is not
// allowed there) or when allocation fails: the call then runs without it and
// its errors are still recorded in its scratch.
uint32_t* device_error_word(hipStream_t s)
{
    const int dev = current_device();
    if (dev < 0)
        return nullptr;
    HostErrorWords& W = host_error_words();
    std::lock_guard<std::mutex> g(W.mu);
    auto it = W.device.find(dev);
    if (it != W.device.end())
        return it->second;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (cs != hipStreamCaptureStatusNone)
        return nullptr;
    void* h = nullptr;
    void* d = nullptr;
    if (hipHostMalloc(&h, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    if (hipHostGetDevicePointer(&d, h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(h);
        return nullptr;
    }
    memset(h, 0, 64);
    W.host[dev] = reinterpret_cast<uint32_t*>(h);
    W.device[dev] = reinterpret_cast<uint32_t*>(d);
    return W.device[dev];
}

}  // namespace

namespace evosort {
evosort_status status_of_error_bits(uint32_t bits)
{
    if (bits == 0)
        return EVOSORT_OK;
    return (bits & kDeviceErrBadSegment) ? EVOSORT_ERR_INVALID_ARG : EVOSORT_ERR_DEVICE_TIMEOUT;
}
}  // namespace evosort

namespace {

// Kernel address of the current device's word if it has been allocated
// already (never allocates).
uint32_t* existing_device_error_word()
{
    const int dev = current_device();
    if (dev < 0)
        return nullptr;
    HostErrorWords& W = host_error_words();
    std::lock_guard<std::mutex> g(W.mu);
    auto it = W.device.find(dev);
    return it == W.device.end() ? nullptr : it->second;
}

// Reads and clears the current device's pending error (EVOSORT_OK if none).
evosort_status take_pending_error()
{
    const int dev = current_device();
    if (dev < 0)
        return EVOSORT_OK;
    HostErrorWords& W = host_error_words();
    uint32_t* h = nullptr;
    {
        std::lock_guard<std::mutex> g(W.mu);
        auto it = W.host.find(dev);
        if (it == W.host.end())
            return EVOSORT_OK;
        h = it->second;
    }
    if (__atomic_load_n(h, __ATOMIC_ACQUIRE) == 0)
        return EVOSORT_OK;
    return status_of_error_bits(__atomic_exchange_n(h, 0u, __ATOMIC_ACQ_REL));
}

constexpr uint32_t kDefaultSpinLimit = 1u << 24;
constexpr uint32_t kDefaultInsertion = 8;
constexpr size_t kAlign = 256;
constexpr int64_t kStatus32Limit = (int64_t)1 << 30;  // 32-bit look-back words hold counts < 2^30
constexpr uint64_t kPrefixMinTiles = 256;  // fewer tiles: pass 0 uses the look-back

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool key_desc(int dtype, KeyDesc* kd, bool* is_int)
{
    switch (dtype) {
    case EVOSORT_INT32:
        *kd = {4, 0x80000000ull, 0};
        *is_int = true;
        return true;
    case EVOSORT_UINT32:
        *kd = {4, 0, 0};
        *is_int = true;
        return true;
    case EVOSORT_FLOAT32:
        *kd = {4, 0x80000000ull, 0xffffffffull};
        *is_int = false;
        return true;
    case EVOSORT_INT64:
        *kd = {8, 0x8000000000000000ull, 0};
        *is_int = true;
        return true;
    case EVOSORT_FLOAT64:
        *kd = {8, 0x8000000000000000ull, ~0ull};
        *is_int = false;
        return true;
    default:
        return false;
    }
}

// --------------------------------------------------------------- profiling --
struct ProfRecord {
    const char* name;
    hipEvent_t start;
    hipEvent_t stop;
};

struct Profiler {
    std::mutex mu;
    bool on = false;
    std::vector<ProfRecord> pending;
    std::vector<hipEvent_t> pool;
    std::vector<std::string> names;
    std::map<std::string, std::pair<uint64_t, double>> totals;

    hipEvent_t get_event()
    {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess)
            return nullptr;
        return e;
    }
};

Profiler& prof()
{
    static Profiler* p = new Profiler();  // never destroyed: events outlive static teardown order
    return *p;
}

// Runs one kernel launch, bracketed by events when profiling is on.
template <class F>
hipError_t timed(const char* name, hipStream_t s, F&& launch)
{
    // Launchers report hipGetLastError(); drop any error an unrelated earlier
    // runtime call left behind so it is not blamed on this launch.
    (void)hipGetLastError();
    Profiler& P = prof();
    bool on;
    {
        std::lock_guard<std::mutex> g(P.mu);
        on = P.on && !t_no_events;
    }
    if (!on)
        return launch();
    hipEvent_t a, b;
    {
        std::lock_guard<std::mutex> g(P.mu);
        a = P.get_event();
        b = P.get_event();
    }
    auto give_back = [&] {
        std::lock_guard<std::mutex> g(P.mu);
        if (a)
            P.pool.push_back(a);
        if (b)
            P.pool.push_back(b);
    };
    if (!a || !b || hipEventRecord(a, s) != hipSuccess) {
        (void)hipGetLastError();
        give_back();  // this launch goes untimed
        return launch();
    }
    const hipError_t e = launch();
    if (hipEventRecord(b, s) != hipSuccess) {
        (void)hipGetLastError();
        give_back();
        return e;
    }
    std::lock_guard<std::mutex> g(P.mu);
    P.pending.push_back({name, a, b});
    return e;
}

// ------------------------------------------------------------------ plan ----
struct Plan {
    evosort_plan_info info;
    KeyDesc kd;
    bool is_int;
    int op;
    int64_t n;
    int vb;  // value or index bytes
    int bits;
    RadixShape shape;
    uint32_t spin_limit;
    uint32_t debug_flags;
    uint32_t t_ins;
    // radix scratch layout (byte offsets into temp)
    size_t off_keys_a, off_keys_b, off_vals, off_hist, off_bases, off_status, off_ctr, off_err, off_blocks, off_live,
        off_done;
    bool prefix0;  // pass 0 takes its tile offsets from the histogram's per-tile counts
    size_t zero_begin, zero_end;
    size_t status_pass_bytes;
    // merge scratch layout
    MergePlan mp;
    size_t off_mkeys, off_mkeys2, off_mvals, off_parts;
    size_t total;
    uint32_t* host_error;  // host-visible error word the kernels also set (null: none)
};

evosort_status check_params(const evosort_params* p)
{
    if (p->struct_size != sizeof(evosort_params))
        return EVOSORT_ERR_INVALID_ARG;
    if (p->algo != EVOSORT_ALGO_AUTO && p->algo != EVOSORT_ALGO_MERGE && p->algo != EVOSORT_ALGO_RADIX)
        return EVOSORT_ERR_INVALID_ARG;
    if (p->digit_bits < 4 || p->digit_bits > 12)
        return EVOSORT_ERR_INVALID_ARG;
    if (p->insertion_threshold < 1 || p->insertion_threshold > 2048)
        return EVOSORT_ERR_INVALID_ARG;
    if ((p->block_threads == 0) != (p->items_per_thread == 0))
        return EVOSORT_ERR_INVALID_ARG;
    if (p->descending > 1 || p->reserved != 0)
        return EVOSORT_ERR_INVALID_ARG;
    return EVOSORT_OK;
}

void default_params(evosort_params* p)
{
    memset(p, 0, sizeof(*p));
    p->struct_size = sizeof(evosort_params);
    p->algo = EVOSORT_ALGO_AUTO;
    p->digit_bits = 8;
    p->insertion_threshold = kDefaultInsertion;
    p->fallback_threshold = (uint64_t)kSmallCapacity;
    p->block_threads = 0;
    p->items_per_thread = 0;
    p->spin_limit = 0;
    p->debug_flags = 0;
}

enum ForcePath { FORCE_NONE = 0, FORCE_RADIX = 1, FORCE_MERGE = 2 };

// The GA table's row for a keys-only sort of n keys of type dtype (the row of
// that key type whose length range lo <= n < hi holds n), or null.
const TunedRow* tuned_row(int dtype, int64_t n)
{
    for (int i = 0; i < kTunedRowCount; ++i) {
        const TunedRow& r = kTunedRows[i];
        if (r.dtype == dtype && n >= r.lo && n < r.hi)
            return &r;
    }
    return nullptr;
}

evosort_status make_plan(int op, int dtype, int64_t n, uint32_t value_bytes, const evosort_params* pin, Plan* P,
                         ForcePath force = FORCE_NONE)
{
    memset(P, 0, sizeof(*P));
    evosort_params p;
    if (pin) {
        p = *pin;
        evosort_status st = check_params(&p);
        if (st != EVOSORT_OK)
            return st;
    } else {
        default_params(&p);
    }
    if (n < 0)
        return EVOSORT_ERR_INVALID_ARG;
    if (op != EVOSORT_OP_SORT && op != EVOSORT_OP_SORT_PAIRS && op != EVOSORT_OP_ARGSORT)
        return EVOSORT_ERR_INVALID_ARG;
    if (!key_desc(dtype, &P->kd, &P->is_int))
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    P->kd.desc = p.descending ? ~0ull : 0ull;
    if (op == EVOSORT_OP_SORT) {
        if (value_bytes != 0)
            return EVOSORT_ERR_INVALID_ARG;
    } else if (value_bytes != 4 && value_bytes != 8) {
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    }
    if (op == EVOSORT_OP_ARGSORT && value_bytes == 4 && n > 0x7fffffffLL)
        return EVOSORT_ERR_INVALID_ARG;

    const int kb = P->kd.bytes;
    const int vb = (int)value_bytes;
    P->op = op;
    P->n = n;
    P->vb = vb;
    P->bits = (int)p.digit_bits;
    P->spin_limit = p.spin_limit ? p.spin_limit : kDefaultSpinLimit;
    P->debug_flags = p.debug_flags;
    P->t_ins = p.insertion_threshold;
    P->shape = p.block_threads ? RadixShape{(int)p.block_threads, (int)p.items_per_thread}
                               : radix_default_shape_for(kb, vb, (int)p.digit_bits, n);
    // Automatic choice (A_code 0) of a keys-only sort with no shape given:
    // where the GA tuner's table has a row for this key type and length, the
    // row's routine replaces the default radix sort (Sec. 4.2, Algorithm 2;
    // the table is compiled in from the tuner's output).
    int tuned_algo = 0;
    if (p.algo == EVOSORT_ALGO_AUTO && op == EVOSORT_OP_SORT && !p.block_threads) {
        if (const TunedRow* row = tuned_row(dtype, n))
            tuned_algo = row->algo;
    }
    const int64_t cap = small_sort_capacity(kb, vb);
    P->info.small_capacity = (uint64_t)cap;
    P->info.digit_bits = p.digit_bits;
    P->info.block_threads = (uint32_t)P->shape.threads;
    P->info.items_per_thread = (uint32_t)P->shape.items;

    // The adaptive partition sort (Sec. 4.3, Algorithm 6), with the readings
    // of the GPU library: the small-array branch is capped by one
    // workgroup's capacity; float keys take the radix branch too; A_code 0
    // means radix unless the tuner's table picked the mergesort for this size
    // class.
    int path;
    if (force == FORCE_RADIX)
        path = EVOSORT_PATH_RADIX;
    else if (force == FORCE_MERGE)
        path = EVOSORT_PATH_MERGE;
    else if (n <= 1)
        path = EVOSORT_PATH_COPY;
    else if ((uint64_t)n < p.fallback_threshold && n <= cap)
        path = EVOSORT_PATH_SMALL;
    else if (p.algo == EVOSORT_ALGO_MERGE || tuned_algo == EVOSORT_ALGO_MERGE)
        path = EVOSORT_PATH_MERGE;
    else
        path = EVOSORT_PATH_RADIX;
    P->info.path = path;

    // Scratch layouts.  Both start with a 256-byte header whose first word is
    // the device error word (evosort_check_device_error reads it there).
    size_t off = 0;
    if (path == EVOSORT_PATH_RADIX) {
        const int passes = (8 * kb + P->bits - 1) / P->bits;
        const int status_bytes = n < kStatus32Limit && !(p.debug_flags & EVOSORT_DEBUG_WIDE_STATUS) ? 4 : 8;
        if (!radix_pass_available(kb, vb, P->bits, P->shape, status_bytes))
            return EVOSORT_ERR_UNSUPPORTED_PARAM;
        const uint64_t tile = (uint64_t)P->shape.threads * P->shape.items;
        const uint64_t tiles = ((uint64_t)n + tile - 1) / tile;
        if (tiles > 0xffffffffull)
            return EVOSORT_ERR_INVALID_ARG;
        const size_t bins = (size_t)1 << P->bits;
        P->info.passes = (uint32_t)passes;
        P->info.status_bytes = (uint32_t)status_bytes;
        P->info.tile_keys = tile;
        P->info.tiles = tiles;
        // zeroed on every call: header (error word, tile counters), histograms, look-back words
        P->zero_begin = 0;
        P->off_err = 0;
        P->off_live = 16;  // the live-pass word (zeroed here, bits set by the scan)
        P->off_done = 20;  // scan workgroups finished
        P->off_ctr = 64;   // 64-bit ticket counters: passes * 8 <= 128 bytes
        off = kAlign;
        P->off_hist = off;
        off = align_up(off + (size_t)passes * bins * 8);
        P->status_pass_bytes = align_up((size_t)tiles * bins * status_bytes);
        P->off_status = off;
        off += (size_t)passes * P->status_pass_bytes;
        P->zero_end = off;
        P->off_bases = off;
        off = align_up(off + (size_t)passes * bins * 8);
        // 8-bit digits, all passes in one histogram launch: pass 0's tile
        // offsets come from per-tile counts and an exclusive scan over tiles
        // Pass 0 takes its tile offsets from a scan over the histogram's
        // per-tile counts, which costs three more launches; with few tiles
        // the look-back is cheaper (int32, ms per sort with / without:
        // 1e5 0.124 / 0.105, 1e6 0.162 / 0.132, 3e6 (163 tiles) 0.204 /
        // 0.175, 1e7 (543 tiles) 0.301 / 0.307).
        P->prefix0 = P->bits == 8 && passes == kb && tiles >= kPrefixMinTiles;
        P->off_blocks = off;
        if (P->prefix0)
            off = align_up(off + (size_t)((tiles + kTilePrefixBlock - 1) / kTilePrefixBlock) * 256 * 8);
        P->off_keys_a = off;
        off = align_up(off + (size_t)n * kb);
        if (op == EVOSORT_OP_ARGSORT) {
            P->off_keys_b = off;
            off = align_up(off + (size_t)n * kb);
        }
        if (vb) {
            P->off_vals = off;
            off = align_up(off + (size_t)n * vb);
        }
    } else if (path == EVOSORT_PATH_MERGE) {
        P->mp = merge_plan(kb, vb, n, P->t_ins);
        P->info.tile_keys = P->mp.block_keys;
        P->info.tiles = P->mp.blocks;
        P->info.merge_rounds = P->mp.rounds;
        P->info.merge_block_run = P->mp.block_run;
        P->off_err = 0;
        off = kAlign;
        P->off_mkeys = off;
        off = align_up(off + (size_t)n * kb);
        if (op == EVOSORT_OP_ARGSORT) {
            P->off_mkeys2 = off;
            off = align_up(off + (size_t)n * kb);
        }
        if (vb) {
            P->off_mvals = off;
            off = align_up(off + (size_t)n * vb);
        }
        P->off_parts = off;
        off = align_up(off + merge_partition_bytes(P->mp));
    } else if (path == EVOSORT_PATH_SMALL) {
        P->off_err = 0;  // the header only: the kernel clears its error word
        off = kAlign;
    }
    P->total = off;
    P->info.temp_bytes = off;
    return EVOSORT_OK;
}

// ------------------------------------------------------------ arg checks ----
bool overlaps(const void* a, size_t an, const void* b, size_t bn)
{
    if (!a || !b || an == 0 || bn == 0)
        return false;
    const uintptr_t x = (uintptr_t)a, y = (uintptr_t)b;
    return x < y + bn && y < x + an;
}

// Distinct buffers must not overlap; pairs listed in `same_ok` may be equal.
evosort_status check_buffers(const void* const* bufs, const size_t* sizes, int count, int same_ok_a1, int same_ok_b1,
                             int same_ok_a2, int same_ok_b2)
{
    for (int i = 0; i < count; ++i)
        for (int j = i + 1; j < count; ++j) {
            if (!bufs[i] || !bufs[j])
                continue;
            const bool ok_pair = (i == same_ok_a1 && j == same_ok_b1) || (i == same_ok_a2 && j == same_ok_b2);
            if (ok_pair && bufs[i] == bufs[j])
                continue;
            if (overlaps(bufs[i], sizes[i], bufs[j], sizes[j]))
                return EVOSORT_ERR_INVALID_ARG;
        }
    return EVOSORT_OK;
}

evosort_status hip_fail(hipError_t e)
{
    t_last_hip = (int)e;
    return EVOSORT_ERR_HIP;
}

}  // namespace

namespace evosort {
evosort_status record_hip_failure(hipError_t e) { return hip_fail(e); }
}  // namespace evosort

namespace {

#define EVOSORT_LAUNCH(name, s, expr)                         \
    do {                                                      \
        hipError_t e_ = timed((name), (s), [&] { return (expr); }); \
        if (e_ != hipSuccess)                                 \
            return hip_fail(e_);                              \
    } while (0)

unsigned char* at(void* temp, size_t off) { return reinterpret_cast<unsigned char*>(temp) + off; }

// ------------------------------------------------------------ radix path ----
// Buffers: the input keys (read only unless sorted in place), the output, and
// one (argsort: two) key buffer(s) in temp; values likewise.  Every pass is
// launched; on the device each pass learns from the scan which passes have a
// digit that varies, skips itself if its digit is constant, and otherwise
// picks its input and output so that the last live pass writes the output
// (RadixRoute).  A final launch does the copy that an odd number of live
// passes sorted in place, or no live pass at all, leaves to do.
evosort_status run_radix(const Plan& P, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                         void* temp, hipStream_t s)
{
    const int kb = P.kd.bytes, vb = P.vb;
    const int passes = (int)P.info.passes;
    const size_t bins = (size_t)1 << P.bits;
    const int64_t n = P.n;
    auto* hist = reinterpret_cast<uint64_t*>(at(temp, P.off_hist));
    auto* bases = reinterpret_cast<uint64_t*>(at(temp, P.off_bases));
    auto* tickets = reinterpret_cast<unsigned long long*>(at(temp, P.off_ctr));
    auto* err = reinterpret_cast<uint32_t*>(at(temp, P.off_err));
    auto* live = reinterpret_cast<uint32_t*>(at(temp, P.off_live));
    auto* done = reinterpret_cast<uint32_t*>(at(temp, P.off_done));

    EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(at(temp, P.zero_begin), P.zero_end - P.zero_begin, s));
    if (P.prefix0) {
        void* counts0 = at(temp, P.off_status);  // pass 0's status words hold its tile prefixes
        EVOSORT_LAUNCH("radix_histogram", s,
                       launch_radix_histogram_tiles(P.kd, keys_in, n, passes, hist, counts0, (int)P.info.status_bytes,
                                                    (uint32_t)P.info.tile_keys, (uint32_t)P.info.tiles, s));
        EVOSORT_LAUNCH("tile_prefix", s,
                       launch_tile_prefix(counts0, (int)P.info.status_bytes, (uint32_t)P.info.tiles,
                                          reinterpret_cast<uint64_t*>(at(temp, P.off_blocks)), s));
    } else {
        EVOSORT_LAUNCH("radix_histogram", s, launch_radix_histogram(P.kd, keys_in, n, P.bits, passes, hist, s));
    }
    EVOSORT_LAUNCH("radix_scan", s, launch_radix_scan(hist, bases, P.bits, passes, live, done, tickets, s));

    const bool argsort = P.op == EVOSORT_OP_ARGSORT;
    const bool pairs = P.op == EVOSORT_OP_SORT_PAIRS;
    RadixRoute r{};
    r.live = live;
    r.passes = (uint32_t)passes;
    r.flags = argsort ? ROUTE_ARGSORT : 0u;
    // sorted in place: the first live pass must not write the output it reads
    if (!argsort && (keys_out == keys_in || (pairs && vals_out == vals_in)))
        r.flags |= ROUTE_COPY_IF_ODD;
    r.keys_in = keys_in;
    r.keys_out = argsort ? nullptr : keys_out;
    r.keys_tmp = at(temp, P.off_keys_a);
    r.keys_tmp2 = argsort ? at(temp, P.off_keys_b) : nullptr;
    r.vals_in = pairs ? vals_in : nullptr;
    r.vals_out = vb ? vals_out : nullptr;
    r.vals_tmp = vb ? at(temp, P.off_vals) : nullptr;

    for (int p = 0; p < passes; ++p) {
        RadixPassArgs a{};
        a.n = n;
        a.shift = (uint32_t)(p * P.bits);
        a.bases = bases + (size_t)p * bins;
        a.status = at(temp, P.off_status + (size_t)p * P.status_pass_bytes);
        a.ticket = tickets + p;
        a.error_word = err;
        a.host_error = P.host_error;
        a.flags = 0;
        if (P.debug_flags & EVOSORT_DEBUG_WITHHOLD_TILE0)
            a.flags |= RADIX_FLAG_WITHHOLD_T0;
        if (p == 0 && P.prefix0)
            a.flags |= RADIX_FLAG_PREFIX;  // pass 0, when live, is the first live pass: it reads the input
        a.spin_limit = P.spin_limit;
        a.tiles = (uint32_t)P.info.tiles;
        a.route = r;
        a.route.pass = (uint32_t)p;
        EVOSORT_LAUNCH("radix_pass", s,
                       launch_radix_pass(P.kd, vb, P.bits, P.shape, (int)P.info.status_bytes, a,
                                         (uint32_t)P.info.tiles, s));
    }
    EVOSORT_LAUNCH("radix_finish", s, launch_radix_finish(r, n, kb, vb, s));
    return EVOSORT_OK;
}

evosort_status run_small(const Plan& P, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                         void* temp, hipStream_t s)
{
    SmallSortArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.n = P.n;
    a.mode = P.op == EVOSORT_OP_SORT ? SMALL_MODE_KEYS
                                     : (P.op == EVOSORT_OP_SORT_PAIRS ? SMALL_MODE_PAIRS : SMALL_MODE_ARGSORT);
    a.error_word = reinterpret_cast<uint32_t*>(at(temp, P.off_err));
    EVOSORT_LAUNCH("small_sort", s, launch_small_sort(P.kd, P.vb, a, s));
    return EVOSORT_OK;
}

evosort_status run_copy(const Plan& P, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                        hipStream_t s)
{
    const size_t n = (size_t)P.n;
    if (P.op == EVOSORT_OP_ARGSORT) {
        if (n == 1) {
            // the one index is 0
            EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(vals_out, (size_t)P.vb, s));
        }
        return EVOSORT_OK;
    }
    EVOSORT_LAUNCH("copy", s, launch_copy(keys_out, keys_in, n * P.kd.bytes, s));
    if (P.op == EVOSORT_OP_SORT_PAIRS)
        EVOSORT_LAUNCH("copy", s, launch_copy(vals_out, vals_in, n * P.vb, s));
    return EVOSORT_OK;
}

evosort_status run_merge(const Plan& P, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                         void* temp, hipStream_t s)
{
    // no device-side error can occur here; clear the scratch's error word
    EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(temp, kAlign, s));
    MergeBuffers b{};
    b.keys_in = keys_in;
    b.keys_out = keys_out;
    b.vals_in = vals_in;
    b.vals_out = vals_out;
    b.keys_tmp = at(temp, P.off_mkeys);
    b.keys_tmp2 = P.op == EVOSORT_OP_ARGSORT ? at(temp, P.off_mkeys2) : nullptr;
    b.vals_tmp = P.vb ? at(temp, P.off_mvals) : nullptr;
    b.parts = reinterpret_cast<int64_t*>(at(temp, P.off_parts));
    b.iota = P.op == EVOSORT_OP_ARGSORT;
    MergeLaunch ml;
    ml.block_sort = [&](const MergeBlockArgs& a) -> hipError_t {
        return timed("merge_block_sort", s, [&] { return launch_merge_block_sort(P.kd, P.vb, P.mp, a, s); });
    };
    ml.partition = [&](const MergeRoundArgs& a) -> hipError_t {
        return timed("merge_partition", s, [&] { return launch_merge_partition(P.kd, P.mp, a, s); });
    };
    ml.merge = [&](const MergeRoundArgs& a) -> hipError_t {
        return timed("merge_round", s, [&] { return launch_merge_round(P.kd, P.vb, P.mp, a, s); });
    };
    hipError_t e = run_merge_sort(P.mp, b, ml);
    if (e != hipSuccess)
        return hip_fail(e);
    return EVOSORT_OK;
}

evosort_status sort_impl(int op, int dtype, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                         uint32_t vb, int64_t n, void* temp, size_t temp_bytes, const evosort_params* p,
                         hipStream_t s, uint32_t* host_error)
{
    Plan P;
    evosort_status st = make_plan(op, dtype, n, vb, p, &P);
    if (st != EVOSORT_OK)
        return st;
    P.host_error = host_error;
    if (n == 0)
        return EVOSORT_OK;
    const size_t kbytes = (size_t)n * P.kd.bytes;
    const size_t vbytes = (size_t)n * vb;
    if (!keys_in)
        return EVOSORT_ERR_INVALID_ARG;
    if (op != EVOSORT_OP_ARGSORT && !keys_out)
        return EVOSORT_ERR_INVALID_ARG;
    if (op == EVOSORT_OP_SORT_PAIRS && (!vals_in || !vals_out))
        return EVOSORT_ERR_INVALID_ARG;
    if (op == EVOSORT_OP_ARGSORT && !vals_out)
        return EVOSORT_ERR_INVALID_ARG;
    if (temp_bytes < P.total)
        return EVOSORT_ERR_TEMP_TOO_SMALL;
    if (P.total > 0 && (!temp || ((uintptr_t)temp & (kAlign - 1))))
        return EVOSORT_ERR_INVALID_ARG;
    // buffers: 0 keys_in, 1 keys_out, 2 vals_in, 3 vals_out, 4 temp
    const void* bufs[5] = {keys_in, op == EVOSORT_OP_ARGSORT ? nullptr : keys_out,
                           op == EVOSORT_OP_SORT_PAIRS ? vals_in : nullptr, op == EVOSORT_OP_SORT ? nullptr : vals_out,
                           P.total ? temp : nullptr};
    const size_t sizes[5] = {kbytes, kbytes, vbytes, vbytes, P.total};
    st = check_buffers(bufs, sizes, 5, 0, 1, 2, 3);
    if (st != EVOSORT_OK)
        return st;
    switch (P.info.path) {
    case EVOSORT_PATH_COPY:
        // n == 1: a temp buffer, if one is given, still gets a clear error word
        if (temp && temp_bytes >= kAlign && !((uintptr_t)temp & (kAlign - 1)))
            EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(temp, kAlign, s));
        return run_copy(P, keys_in, keys_out, vals_in, vals_out, s);
    case EVOSORT_PATH_SMALL:
        return run_small(P, keys_in, keys_out, vals_in, vals_out, temp, s);
    case EVOSORT_PATH_RADIX:
        return run_radix(P, keys_in, keys_out, vals_in, vals_out, temp, s);
    case EVOSORT_PATH_MERGE:
        return run_merge(P, keys_in, keys_out, vals_in, vals_out, temp, s);
    default:
        return EVOSORT_ERR_INVALID_ARG;
    }
}

// A public sort call: reports a pending device-side error of an earlier call
// first, then runs with the device's host-visible error word.
evosort_status sort_common(int op, int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                           void* vals_out, uint32_t vb, int64_t n, void* temp, size_t temp_bytes,
                           const evosort_params* p, void* stream)
{
    const evosort_status pending = take_pending_error();
    if (pending != EVOSORT_OK)
        return pending;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return sort_impl(op, dtype, keys_in, keys_out, vals_in, vals_out, vb, n, temp, temp_bytes, p, s,
                     device_error_word(s));
}


// ------------------------------------------------------- segmented sort ----
// Scratch of a batched call: the 256-byte header (error word, SegCounters),
// the class lists, the large-segment table, the tile -> segment map, the
// large segments' histograms and bases, the look-back words of every pass,
// and one key (and value) buffer for the passes.  Only the header is zeroed
// by the host sequence; histograms and look-back words are zeroed on the
// device for the segments and tiles in use.
struct SegPlan {
    KeyDesc kd;
    int vb;
    int64_t n, nseg;
    RadixShape shape;
    uint32_t tile_keys;
    int passes;
    int classes;
    int64_t caps[kSegMaxClasses];
    int64_t block_limit;
    uint64_t nlarge_max, tiles_max;
    uint32_t spin_limit, debug_flags;
    size_t off_ctr, off_lists, off_large, off_tile_slot, off_hist, off_bases, off_status, status_pass_bytes,
        off_keys, off_vals, total;
};

constexpr uint32_t kSegHistGroup = 8;  // tiles per histogram workgroup

evosort_status make_seg_plan(int dtype, int64_t n, int64_t nseg, uint32_t value_bytes, const evosort_params* pin,
                             SegPlan* S)
{
    memset(S, 0, sizeof(*S));
    evosort_params p;
    if (pin) {
        p = *pin;
        evosort_status st = check_params(&p);
        if (st != EVOSORT_OK)
            return st;
    } else {
        default_params(&p);
    }
    bool is_int;
    if (!key_desc(dtype, &S->kd, &is_int))
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    S->kd.desc = p.descending ? ~0ull : 0ull;
    if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8)
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    if (n < 0 || nseg < 0 || nseg >= ((int64_t)1 << 32) - 1)
        return EVOSORT_ERR_INVALID_ARG;
    if (p.digit_bits != (uint32_t)kSegBits || p.algo == EVOSORT_ALGO_MERGE)
        return EVOSORT_ERR_UNSUPPORTED_PARAM;
    const int kb = S->kd.bytes, vb = (int)value_bytes, rb = kb + vb;
    S->vb = vb;
    S->n = n;
    S->nseg = nseg;
    S->shape = p.block_threads ? RadixShape{(int)p.block_threads, (int)p.items_per_thread} : seg_default_shape(kb, vb);
    if (!seg_pass_available(kb, vb, S->shape))
        return EVOSORT_ERR_UNSUPPORTED_PARAM;
    S->tile_keys = (uint32_t)(S->shape.threads * S->shape.items);
    S->passes = (8 * kb) / kSegBits;
    S->classes = seg_class_count(rb);
    for (int c = 0; c < S->classes; ++c)
        S->caps[c] = seg_class_capacity(rb, c);
    const int64_t cap_max = seg_block_capacity(rb);
    S->block_limit = p.fallback_threshold < (uint64_t)cap_max + 1 ? (int64_t)p.fallback_threshold : cap_max + 1;
    S->spin_limit = p.spin_limit ? p.spin_limit : kDefaultSpinLimit;
    S->debug_flags = p.debug_flags;
    // Bounds from n and nseg alone: large segments hold >= max(block_limit, 1)
    // keys; each adds at most one partial tile.
    const int64_t least = S->block_limit > 1 ? S->block_limit : 1;
    S->nlarge_max = (uint64_t)(n / least < nseg ? n / least : nseg);
    S->tiles_max = (uint64_t)n / S->tile_keys + S->nlarge_max;
    if (S->tiles_max > 0xffffffffull)
        return EVOSORT_ERR_INVALID_ARG;

    size_t off = kAlign;  // header: error word at 0, counters at 16
    S->off_ctr = 16;
    static_assert(16 + sizeof(SegCounters) <= kAlign, "counters fit in the header");
    S->off_lists = off;
    off = align_up(off + (size_t)(S->classes + 1) * (size_t)nseg * 4);
    S->off_large = off;
    off = align_up(off + (size_t)S->nlarge_max * sizeof(SegLarge));
    S->off_tile_slot = off;
    off = align_up(off + (size_t)S->tiles_max * 4);
    const size_t slot_words = (size_t)S->passes * kSegBins;
    S->off_hist = off;
    off = align_up(off + (size_t)S->nlarge_max * slot_words * 4);
    S->off_bases = off;
    off = align_up(off + (size_t)S->nlarge_max * slot_words * 8);
    S->status_pass_bytes = align_up((size_t)S->tiles_max * kSegBins * 4);
    S->off_status = off;
    off += (size_t)S->passes * S->status_pass_bytes;
    S->off_keys = off;
    off = align_up(off + (size_t)n * kb);
    if (vb) {
        S->off_vals = off;
        off = align_up(off + (size_t)n * vb);
    }
    S->total = off;
    return EVOSORT_OK;
}

// A second stream per device for the short segments of a batched call, so
// that their one-workgroup sorts (latency-bound) run beside the long
// segments' passes (bandwidth-bound) on the caller's stream.  The caller's
// stream forks to it after the classification and joins it at the end, with
// events, so the call stays one capturable sequence (a graph gets two
// branches).  Created on first use and kept; calls that fork hold `mu` from
// the fork to the join so the events are not re-recorded in between.
struct SideStream {
    hipStream_t stream = nullptr;
    hipEvent_t fork = nullptr, join = nullptr;
};
struct SideStreams {
    std::mutex mu;
    std::map<int, SideStream> per_device;
};
SideStreams& side_streams()
{
    static SideStreams* s = new SideStreams();  // never destroyed: streams outlive static teardown order
    return *s;
}
// Returns false (and no side stream) if one cannot be created; the caller
// then runs everything on its own stream.
bool get_side_stream(SideStream* out)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    SideStreams& S = side_streams();
    auto it = S.per_device.find(dev);
    if (it == S.per_device.end()) {
        SideStream ss;
        if (hipStreamCreateWithFlags(&ss.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ss.fork, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&ss.join, hipEventDisableTiming) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        it = S.per_device.emplace(dev, ss).first;
    }
    *out = it->second;
    return true;
}

evosort_status run_segmented(const SegPlan& S, const void* keys_in, void* keys_out, const void* vals_in,
                             void* vals_out, const int64_t* offsets, void* temp, hipStream_t s,
                             uint32_t* host_error)
{
    auto* ctr = reinterpret_cast<SegCounters*>(at(temp, S.off_ctr));
    auto* err = reinterpret_cast<uint32_t*>(at(temp, 0));
    auto* lists = reinterpret_cast<uint32_t*>(at(temp, S.off_lists));
    auto* large = reinterpret_cast<SegLarge*>(at(temp, S.off_large));
    auto* tile_slot = reinterpret_cast<uint32_t*>(at(temp, S.off_tile_slot));
    auto* hist = reinterpret_cast<uint32_t*>(at(temp, S.off_hist));
    auto* bases = reinterpret_cast<uint64_t*>(at(temp, S.off_bases));
    const size_t slot_words = (size_t)S.passes * kSegBins;

    EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(temp, kAlign, s));
    if (S.nseg == 0)
        return EVOSORT_OK;

    SegClassifyArgs ca{};
    ca.offsets = offsets;
    ca.nseg = S.nseg;
    ca.n = S.n;
    ca.block_limit = S.block_limit;
    ca.classes = S.classes;
    for (int c = 0; c < S.classes; ++c)
        ca.cap[c] = S.caps[c];
    ca.tile_keys = S.tile_keys;
    ca.ctr = ctr;
    ca.lists = lists;
    ca.large = large;
    ca.error_word = err;
    ca.host_error = host_error;
    EVOSORT_LAUNCH("seg_classify", s, launch_seg_classify(ca, s));

    // large segments: histograms and bases
    const uint32_t slot_grid = (uint32_t)(S.nlarge_max < 2048 ? S.nlarge_max : 2048);
    SegLargeArgs la{};
    la.nlarge = &ctr->class_count[kSegMaxClasses];
    la.large = large;
    la.tile_slot = tile_slot;
    la.hist = hist;
    la.bases = bases;
    la.passes = S.passes;
    if (S.nlarge_max > 0) {
        EVOSORT_LAUNCH("seg_setup", s, launch_seg_setup(la, S.tile_keys, slot_grid, s));
        SegHistArgs ha{};
        ha.keys = keys_in;
        ha.tile_count = &ctr->tile_count;
        ha.large = large;
        ha.tile_slot = tile_slot;
        ha.hist = hist;
        ha.status = reinterpret_cast<uint32_t*>(at(temp, S.off_status));
        ha.status_pass_words = S.status_pass_bytes / 4;
        ha.tile_keys = S.tile_keys;
        ha.group = kSegHistGroup;
        ha.passes = S.passes;
        const uint32_t hist_grid = (uint32_t)((S.tiles_max + kSegHistGroup - 1) / kSegHistGroup);
        EVOSORT_LAUNCH("seg_histogram", s, launch_seg_histogram(S.kd, ha, hist_grid, s));
        EVOSORT_LAUNCH("seg_scan", s, launch_seg_scan(la, slot_grid, s));
    }

    // small segments: one workgroup each, per class; on the side stream when
    // there are long segments too
    bool has_small = false;
    for (int c = 0; c < S.classes; ++c)
        has_small = has_small || (c == 0 ? 1 : S.caps[c - 1] + 1) < S.block_limit;
    std::unique_lock<std::mutex> side_lock(side_streams().mu, std::defer_lock);
    SideStream side{};
    bool forked = false;
    if (has_small && S.nlarge_max > 0) {
        side_lock.lock();
        if (get_side_stream(&side)) {
            if (hipEventRecord(side.fork, s) != hipSuccess || hipStreamWaitEvent(side.stream, side.fork, 0) != hipSuccess)
                return hip_fail(hipGetLastError());
            forked = true;
        } else {
            side_lock.unlock();
        }
    }
    const hipStream_t ss = forked ? side.stream : s;
    for (int c = 0; c < S.classes; ++c) {
        // class c holds segments longer than class c-1's capacity
        const int64_t least = c == 0 ? 1 : S.caps[c - 1] + 1;
        if (least >= S.block_limit)
            break;
        const int64_t bound = S.n / least < S.nseg ? S.n / least : S.nseg;
        SegBlockArgs ba{};
        ba.keys_in = keys_in;
        ba.keys_out = keys_out;
        ba.vals_in = vals_in;
        ba.vals_out = vals_out;
        ba.offsets = offsets;
        ba.list = lists + (size_t)c * S.nseg;
        ba.count = &ctr->class_count[c];
        ba.ticket = &ctr->class_ticket[c];
        EVOSORT_LAUNCH("seg_block_sort", ss,
                       launch_seg_block_sort(S.kd, S.vb, c, ba, (uint32_t)(bound < 0xffffffffLL ? bound : 0xffffffffLL),
                                             ss));
    }
    if (forked && hipEventRecord(side.join, side.stream) != hipSuccess)
        return hip_fail(hipGetLastError());

    // large segments: the passes alternate between temp and the output so
    // that the last (odd-numbered) pass writes the output
    if (S.nlarge_max > 0) {
        void* tk = at(temp, S.off_keys);
        void* tv = S.vb ? at(temp, S.off_vals) : nullptr;
        for (int p = 0; p < S.passes; ++p) {
            SegPassArgs pa{};
            RadixPassArgs& a = pa.base;
            const bool to_temp = (p & 1) == 0;
            a.keys_in = p == 0 ? keys_in : (to_temp ? keys_out : tk);
            a.keys_out = to_temp ? tk : keys_out;
            if (S.vb) {
                a.vals_in = p == 0 ? vals_in : (to_temp ? vals_out : tv);
                a.vals_out = to_temp ? tv : vals_out;
            }
            a.n = S.n;
            a.shift = (uint32_t)(p * kSegBits);
            a.bases = bases + (size_t)p * kSegBins;
            a.status = at(temp, S.off_status + (size_t)p * S.status_pass_bytes);
            a.tile_counter = &ctr->pass_ticket[p];
            a.error_word = err;
            a.host_error = host_error;
            a.flags = (S.debug_flags & EVOSORT_DEBUG_WITHHOLD_TILE0) ? RADIX_FLAG_WITHHOLD_T0 : 0u;
            a.spin_limit = S.spin_limit;
            a.tiles = 0;
            pa.tile_slot = tile_slot;
            pa.large = large;
            pa.tile_count = &ctr->tile_count;
            pa.slot_stride = (uint32_t)slot_words;
            EVOSORT_LAUNCH("seg_radix_pass", s,
                           launch_seg_radix_pass(S.kd, S.vb, S.shape, pa, (uint32_t)S.tiles_max, s));
        }
    }
    if (forked && hipStreamWaitEvent(s, side.join, 0) != hipSuccess)  // join: the caller's stream waits
        return hip_fail(hipGetLastError());
    return EVOSORT_OK;
}

evosort_status segmented_impl(int dtype, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                              uint32_t vb, int64_t n, const int64_t* offsets, int64_t nseg, void* temp,
                              size_t temp_bytes, const evosort_params* p, hipStream_t s, uint32_t* host_error)
{
    SegPlan S;
    evosort_status st = make_seg_plan(dtype, n, nseg, vb, p, &S);
    if (st != EVOSORT_OK)
        return st;
    if (nseg > 0 && !offsets)
        return EVOSORT_ERR_INVALID_ARG;
    if (n > 0 && (!keys_in || !keys_out || (vb && (!vals_in || !vals_out))))
        return EVOSORT_ERR_INVALID_ARG;
    if (temp_bytes < S.total)
        return EVOSORT_ERR_TEMP_TOO_SMALL;
    if (!temp || ((uintptr_t)temp & (kAlign - 1)))
        return EVOSORT_ERR_INVALID_ARG;
    const size_t kbytes = (size_t)n * S.kd.bytes, vbytes = (size_t)n * vb;
    // buffers: 0 keys_in, 1 keys_out, 2 vals_in, 3 vals_out, 4 temp, 5 offsets
    const void* bufs[6] = {keys_in, keys_out, vb ? vals_in : nullptr, vb ? vals_out : nullptr, temp, offsets};
    const size_t sizes[6] = {kbytes, kbytes, vbytes, vbytes, S.total, (size_t)(nseg + 1) * 8};
    st = check_buffers(bufs, sizes, 6, 0, 1, 2, 3);
    if (st != EVOSORT_OK)
        return st;
    return run_segmented(S, keys_in, keys_out, vals_in, vals_out, offsets, temp, s, host_error);
}

evosort_status segmented_common(int dtype, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                                uint32_t vb, int64_t n, const int64_t* offsets, int64_t nseg, void* temp,
                                size_t temp_bytes, const evosort_params* p, void* stream)
{
    const evosort_status pending = take_pending_error();
    if (pending != EVOSORT_OK)
        return pending;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    return segmented_impl(dtype, keys_in, keys_out, vals_in, vals_out, vb, n, offsets, nseg, temp, temp_bytes, p, s,
                          device_error_word(s));
}
}  // namespace

namespace evosort {
evosort_status server_sort(int dtype, const void* keys_in, void* keys_out, int64_t n, void* temp,
                           size_t temp_bytes, const evosort_params* p, hipStream_t s, uint32_t* host_error)
{
    return sort_impl(EVOSORT_OP_SORT, dtype, keys_in, keys_out, nullptr, nullptr, 0, n, temp, temp_bytes, p, s,
                     host_error);
}

evosort_status sort_in_scratch(int dtype, const void* keys_in, void* keys_out, int64_t n, const evosort_params* p,
                               hipStream_t s, void* scratch, size_t scratch_bytes)
{
    const evosort_status pending = take_pending_error();
    if (pending != EVOSORT_OK)
        return pending;
    Plan P;
    const evosort_status st = make_plan(EVOSORT_OP_SORT, dtype, n, 0, p, &P);
    if (st != EVOSORT_OK)
        return st;
    if (P.total > scratch_bytes)
        return EVOSORT_ERR_TEMP_TOO_SMALL;
    t_no_events = true;
    const evosort_status r = sort_impl(EVOSORT_OP_SORT, dtype, keys_in, keys_out, nullptr, nullptr, 0, n, scratch,
                                       scratch_bytes, p, s, existing_device_error_word());
    t_no_events = false;
    return r;
}

evosort_status server_segmented_sort(int dtype, const void* keys_in, void* keys_out, int64_t n,
                                     const int64_t* offsets, int64_t nseg, void* temp, size_t temp_bytes,
                                     const evosort_params* p, hipStream_t s, uint32_t* host_error)
{
    return segmented_impl(dtype, keys_in, keys_out, nullptr, nullptr, 0, n, offsets, nseg, temp, temp_bytes, p, s,
                          host_error);
}
}  // namespace evosort

// ===================================================================== ABI ===
extern "C" {

void evosort_default_params(evosort_params* p)
{
    if (p)
        default_params(p);
}

evosort_status evosort_temp_bytes(int op, int dtype, int64_t n, uint32_t value_bytes, const evosort_params* p,
                                  size_t* out_bytes)
{
    if (!out_bytes)
        return EVOSORT_ERR_INVALID_ARG;
    Plan P;
    evosort_status st = make_plan(op, dtype, n, value_bytes, p, &P);
    if (st != EVOSORT_OK)
        return st;
    // Step functions of both routines run on the same scratch.
    Plan R, M;
    size_t need = P.total;
    if (n > 0 && make_plan(op, dtype, n, value_bytes, p, &R, FORCE_RADIX) == EVOSORT_OK && R.total > need)
        need = R.total;
    if (n > 0 && make_plan(op, dtype, n, value_bytes, p, &M, FORCE_MERGE) == EVOSORT_OK && M.total > need)
        need = M.total;
    *out_bytes = need;
    return EVOSORT_OK;
}

evosort_status evosort_plan(int op, int dtype, int64_t n, uint32_t value_bytes, const evosort_params* p,
                            evosort_plan_info* out)
{
    if (!out)
        return EVOSORT_ERR_INVALID_ARG;
    Plan P;
    evosort_status st = make_plan(op, dtype, n, value_bytes, p, &P);
    if (st != EVOSORT_OK)
        return st;
    *out = P.info;
    size_t need = 0;
    evosort_temp_bytes(op, dtype, n, value_bytes, p, &need);
    out->temp_bytes = need;
    return EVOSORT_OK;
}

evosort_status evosort_sort(int dtype, const void* keys_in, void* keys_out, int64_t n, void* temp, size_t temp_bytes,
                            const evosort_params* p, void* stream)
{
    return sort_common(EVOSORT_OP_SORT, dtype, keys_in, keys_out, nullptr, nullptr, 0, n, temp, temp_bytes, p,
                       stream);
}

evosort_status evosort_sort_pairs(int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                                  void* vals_out, uint32_t value_bytes, int64_t n, void* temp, size_t temp_bytes,
                                  const evosort_params* p, void* stream)
{
    return sort_common(EVOSORT_OP_SORT_PAIRS, dtype, keys_in, keys_out, vals_in, vals_out, value_bytes, n, temp,
                       temp_bytes, p, stream);
}

evosort_status evosort_argsort(int dtype, const void* keys_in, void* idx_out, uint32_t index_bytes, int64_t n,
                               void* temp, size_t temp_bytes, const evosort_params* p, void* stream)
{
    return sort_common(EVOSORT_OP_ARGSORT, dtype, keys_in, nullptr, nullptr, idx_out, index_bytes, n, temp,
                       temp_bytes, p, stream);
}

evosort_status evosort_radix_histogram(int dtype, const void* keys, int64_t n, uint32_t digit_bits,
                                       uint64_t* hist_out, uint64_t* bases_out, void* temp, size_t temp_bytes,
                                       void* stream)
{
    (void)temp;
    (void)temp_bytes;
    KeyDesc kd;
    bool is_int;
    if (!key_desc(dtype, &kd, &is_int))
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    if (n < 0 || digit_bits < 4 || digit_bits > 12 || !hist_out || (n > 0 && !keys))
        return EVOSORT_ERR_INVALID_ARG;
    const int bits = (int)digit_bits;
    const int passes = (8 * kd.bytes + bits - 1) / bits;
    const size_t row_bytes = (size_t)passes * ((size_t)1 << bits) * 8;
    if (overlaps(hist_out, row_bytes, keys, (size_t)n * kd.bytes) ||
        (bases_out && (overlaps(bases_out, row_bytes, keys, (size_t)n * kd.bytes) ||
                       overlaps(bases_out, row_bytes, hist_out, row_bytes))))
        return EVOSORT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // hist_out is zeroed and filled directly (row_bytes is a multiple of 16)
    EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(hist_out, row_bytes, s));
    if (n > 0)
        EVOSORT_LAUNCH("radix_histogram", s, launch_radix_histogram(kd, keys, n, bits, passes, hist_out, s));
    if (bases_out)
        EVOSORT_LAUNCH("radix_scan", s, launch_radix_scan(hist_out, bases_out, bits, passes, nullptr, nullptr, nullptr,
                                                          s));
    return EVOSORT_OK;
}

evosort_status evosort_radix_pass(int dtype, const void* keys_in, void* keys_out, const void* vals_in, void* vals_out,
                                  uint32_t value_bytes, int64_t n, uint32_t pass, void* temp, size_t temp_bytes,
                                  const evosort_params* p, void* stream)
{
    const int op = value_bytes ? EVOSORT_OP_SORT_PAIRS : EVOSORT_OP_SORT;
    const evosort_status pending = take_pending_error();
    if (pending != EVOSORT_OK)
        return pending;
    Plan P;
    evosort_status st = make_plan(op, dtype, n, value_bytes, p, &P, FORCE_RADIX);
    if (st != EVOSORT_OK)
        return st;
    if (pass >= P.info.passes)
        return EVOSORT_ERR_INVALID_ARG;
    if (n == 0)
        return EVOSORT_OK;
    if (!keys_in || !keys_out || (value_bytes && (!vals_in || !vals_out)))
        return EVOSORT_ERR_INVALID_ARG;
    if (temp_bytes < P.total)
        return EVOSORT_ERR_TEMP_TOO_SMALL;
    if (!temp || ((uintptr_t)temp & (kAlign - 1)))
        return EVOSORT_ERR_INVALID_ARG;
    const size_t kbytes = (size_t)n * P.kd.bytes, vbytes = (size_t)n * value_bytes;
    const void* bufs[5] = {keys_in, keys_out, value_bytes ? vals_in : nullptr, value_bytes ? vals_out : nullptr, temp};
    const size_t sizes[5] = {kbytes, kbytes, vbytes, vbytes, P.total};
    st = check_buffers(bufs, sizes, 5, -1, -1, -1, -1);
    if (st != EVOSORT_OK)
        return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const size_t bins = (size_t)1 << P.bits;
    auto* hist = reinterpret_cast<uint64_t*>(at(temp, P.off_hist));
    auto* bases = reinterpret_cast<uint64_t*>(at(temp, P.off_bases));
    EVOSORT_LAUNCH("fill_zero", s, launch_fill_zero(at(temp, P.zero_begin), P.zero_end - P.zero_begin, s));
    EVOSORT_LAUNCH("radix_histogram", s,
                   launch_radix_histogram(P.kd, keys_in, n, P.bits, (int)P.info.passes, hist, s));
    EVOSORT_LAUNCH("radix_scan", s,
                   launch_radix_scan(hist, bases, P.bits, (int)P.info.passes, nullptr, nullptr, nullptr, s));
    RadixPassArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.n = n;
    a.shift = pass * (uint32_t)P.bits;
    a.bases = bases + (size_t)pass * bins;
    a.status = at(temp, P.off_status);
    a.ticket = reinterpret_cast<unsigned long long*>(at(temp, P.off_ctr));  // zeroed: no route code
    a.error_word = reinterpret_cast<uint32_t*>(at(temp, P.off_err));
    a.host_error = device_error_word(s);
    a.flags = (P.debug_flags & EVOSORT_DEBUG_WITHHOLD_TILE0) ? RADIX_FLAG_WITHHOLD_T0 : 0u;
    a.spin_limit = P.spin_limit;
    a.tiles = (uint32_t)P.info.tiles;
    EVOSORT_LAUNCH("radix_pass", s,
                   launch_radix_pass(P.kd, (int)value_bytes, P.bits, P.shape, (int)P.info.status_bytes, a,
                                     (uint32_t)P.info.tiles, s));
    return EVOSORT_OK;
}

evosort_status evosort_merge_block_sort(int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                                        void* vals_out, uint32_t value_bytes, int64_t n, const evosort_params* p,
                                        int64_t* run_out, void* stream)
{
    const int op = value_bytes ? EVOSORT_OP_SORT_PAIRS : EVOSORT_OP_SORT;
    Plan P;
    evosort_status st = make_plan(op, dtype, n, value_bytes, p, &P, FORCE_MERGE);
    if (st != EVOSORT_OK)
        return st;
    if (run_out)
        *run_out = (int64_t)P.mp.block_run;
    if (n == 0)
        return EVOSORT_OK;
    if (!keys_in || !keys_out || (value_bytes && (!vals_in || !vals_out)))
        return EVOSORT_ERR_INVALID_ARG;
    const size_t kbytes = (size_t)n * P.kd.bytes, vbytes = (size_t)n * value_bytes;
    const void* bufs[4] = {keys_in, keys_out, value_bytes ? vals_in : nullptr, value_bytes ? vals_out : nullptr};
    const size_t sizes[4] = {kbytes, kbytes, vbytes, vbytes};
    st = check_buffers(bufs, sizes, 4, -1, -1, -1, -1);
    if (st != EVOSORT_OK)
        return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MergeBlockArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.n = n;
    a.iota = false;
    a.skip_keys = false;
    EVOSORT_LAUNCH("merge_block_sort", s, launch_merge_block_sort(P.kd, (int)value_bytes, P.mp, a, s));
    return EVOSORT_OK;
}

evosort_status evosort_merge_round(int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                                   void* vals_out, uint32_t value_bytes, int64_t n, int64_t run, void* temp,
                                   size_t temp_bytes, void* stream)
{
    const int op = value_bytes ? EVOSORT_OP_SORT_PAIRS : EVOSORT_OP_SORT;
    Plan P;
    evosort_status st = make_plan(op, dtype, n, value_bytes, nullptr, &P, FORCE_MERGE);
    if (st != EVOSORT_OK)
        return st;
    if (run < 1)
        return EVOSORT_ERR_INVALID_ARG;
    if (n == 0)
        return EVOSORT_OK;
    if (!keys_in || !keys_out || (value_bytes && (!vals_in || !vals_out)))
        return EVOSORT_ERR_INVALID_ARG;
    // This step only needs the partition entries of its own round, placed
    // right after the header.
    P.mp.max_parts = merge_round_parts(P.mp, run);
    P.off_parts = kAlign;
    P.total = P.off_parts + merge_partition_bytes(P.mp);
    if (temp_bytes < P.total)
        return EVOSORT_ERR_TEMP_TOO_SMALL;
    if (!temp || ((uintptr_t)temp & (kAlign - 1)))
        return EVOSORT_ERR_INVALID_ARG;
    const size_t kbytes = (size_t)n * P.kd.bytes, vbytes = (size_t)n * value_bytes;
    const void* bufs[5] = {keys_in, keys_out, value_bytes ? vals_in : nullptr, value_bytes ? vals_out : nullptr, temp};
    const size_t sizes[5] = {kbytes, kbytes, vbytes, vbytes, P.total};
    st = check_buffers(bufs, sizes, 5, -1, -1, -1, -1);
    if (st != EVOSORT_OK)
        return st;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    MergeRoundArgs a{};
    a.keys_in = keys_in;
    a.keys_out = keys_out;
    a.vals_in = vals_in;
    a.vals_out = vals_out;
    a.n = n;
    a.run = run;
    a.parts = reinterpret_cast<int64_t*>(at(temp, P.off_parts));
    a.skip_keys = false;
    EVOSORT_LAUNCH("merge_partition", s, launch_merge_partition(P.kd, P.mp, a, s));
    EVOSORT_LAUNCH("merge_round", s, launch_merge_round(P.kd, (int)value_bytes, P.mp, a, s));
    return EVOSORT_OK;
}

evosort_status evosort_segmented_temp_bytes(int dtype, int64_t n, int64_t nseg, uint32_t value_bytes,
                                            const evosort_params* p, size_t* out_bytes)
{
    if (!out_bytes)
        return EVOSORT_ERR_INVALID_ARG;
    SegPlan S;
    evosort_status st = make_seg_plan(dtype, n, nseg, value_bytes, p, &S);
    if (st != EVOSORT_OK)
        return st;
    *out_bytes = S.total;
    return EVOSORT_OK;
}

evosort_status evosort_segmented_sort(int dtype, const void* keys_in, void* keys_out, int64_t n,
                                      const int64_t* offsets, int64_t nseg, void* temp, size_t temp_bytes,
                                      const evosort_params* p, void* stream)
{
    return segmented_common(dtype, keys_in, keys_out, nullptr, nullptr, 0, n, offsets, nseg, temp, temp_bytes, p,
                            stream);
}

evosort_status evosort_segmented_sort_pairs(int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                                            void* vals_out, uint32_t value_bytes, int64_t n,
                                            const int64_t* offsets, int64_t nseg, void* temp, size_t temp_bytes,
                                            const evosort_params* p, void* stream)
{
    if (value_bytes != 4 && value_bytes != 8)
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    return segmented_common(dtype, keys_in, keys_out, vals_in, vals_out, value_bytes, n, offsets, nseg, temp,
                            temp_bytes, p, stream);
}

evosort_status evosort_segmented_capacity(int dtype, uint32_t value_bytes, int64_t* out_keys)
{
    KeyDesc kd;
    bool is_int;
    if (!out_keys)
        return EVOSORT_ERR_INVALID_ARG;
    if (!key_desc(dtype, &kd, &is_int) || (value_bytes != 0 && value_bytes != 4 && value_bytes != 8))
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    *out_keys = seg_block_capacity(kd.bytes + (int)value_bytes);
    return EVOSORT_OK;
}

evosort_status evosort_segmented_stats(const void* temp, size_t temp_bytes, uint32_t* class_counts, uint32_t* tiles,
                                       void* stream)
{
    if (!temp || temp_bytes < kAlign)
        return EVOSORT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e);
    SegCounters c;
    e = hipMemcpy(&c, reinterpret_cast<const unsigned char*>(temp) + 16, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(e);
    if (class_counts)
        for (int i = 0; i <= kSegMaxClasses; ++i)
            class_counts[i] = c.class_count[i];
    if (tiles)
        *tiles = c.tile_count;
    return EVOSORT_OK;
}

evosort_status evosort_sort_each(int dtype, const void* keys_in, void* keys_out, const void* vals_in,
                                 void* vals_out, uint32_t value_bytes, const int64_t* host_offsets, int64_t nseg,
                                 void* temp, size_t temp_bytes, const evosort_params* p, void* stream)
{
    KeyDesc kd;
    bool is_int;
    if (!key_desc(dtype, &kd, &is_int))
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    if (value_bytes != 0 && value_bytes != 4 && value_bytes != 8)
        return EVOSORT_ERR_UNSUPPORTED_DTYPE;
    if (nseg < 0 || (nseg > 0 && !host_offsets))
        return EVOSORT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < nseg; ++i)
        if (host_offsets[i] < 0 || host_offsets[i + 1] < host_offsets[i])
            return EVOSORT_ERR_INVALID_ARG;
    for (int64_t i = 0; i < nseg; ++i) {
        const int64_t b = host_offsets[i], len = host_offsets[i + 1] - b;
        if (len == 0)
            continue;
        const unsigned char* ki = reinterpret_cast<const unsigned char*>(keys_in) + (size_t)b * kd.bytes;
        unsigned char* ko = reinterpret_cast<unsigned char*>(keys_out) + (size_t)b * kd.bytes;
        evosort_status st;
        if (value_bytes == 0) {
            st = sort_common(EVOSORT_OP_SORT, dtype, ki, ko, nullptr, nullptr, 0, len, temp, temp_bytes, p, stream);
        } else {
            const unsigned char* vi = reinterpret_cast<const unsigned char*>(vals_in) + (size_t)b * value_bytes;
            unsigned char* vo = reinterpret_cast<unsigned char*>(vals_out) + (size_t)b * value_bytes;
            st = sort_common(EVOSORT_OP_SORT_PAIRS, dtype, ki, ko, vi, vo, value_bytes, len, temp, temp_bytes, p,
                             stream);
        }
        if (st != EVOSORT_OK)
            return st;
    }
    return EVOSORT_OK;
}

const char* evosort_status_string(int status)
{
    switch (status) {
    case EVOSORT_OK:
        return "ok";
    case EVOSORT_ERR_INVALID_ARG:
        return "invalid argument";
    case EVOSORT_ERR_UNSUPPORTED_DTYPE:
        return "unsupported key, value or index type";
    case EVOSORT_ERR_UNSUPPORTED_PARAM:
        return "unsupported parameter combination (e.g. a tile shape that is not compiled in)";
    case EVOSORT_ERR_TEMP_TOO_SMALL:
        return "temp buffer smaller than evosort_temp_bytes()";
    case EVOSORT_ERR_HIP:
        return "HIP error (see evosort_last_hip_error)";
    case EVOSORT_ERR_DEVICE_TIMEOUT:
        return "a device-side wait ran out of its spin limit";
    case EVOSORT_ERR_OVER_BUDGET:
        return "request needs more HBM than the server's whole budget";
    case EVOSORT_ERR_PENDING:
        return "request not finished yet";
    default:
        return "unknown status";
    }
}

int evosort_last_hip_error(void) { return t_last_hip; }

#ifndef EVOSORT_SOURCE_HASH
#error "the build passes -DEVOSORT_SOURCE_HASH=<hash of the sources>"
#endif
const char* evosort_build_id(void) { return EVOSORT_SOURCE_HASH; }

evosort_status evosort_check_device_error(const void* temp, size_t temp_bytes, void* stream)
{
    // Every radix, mergesort and segmented scratch layout starts with the
    // error word.
    if (!temp || temp_bytes < 4)
        return EVOSORT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess)
        return hip_fail(e);
    uint32_t word = 0;
    e = hipMemcpy(&word, temp, 4, hipMemcpyDeviceToHost);
    if (e != hipSuccess)
        return hip_fail(e);
    if (word != 0)
        (void)take_pending_error();  // this failure is now reported; the next call need not repeat it
    return status_of_error_bits(word);
}

evosort_status evosort_stream_copy(void* dst, const void* src, size_t bytes, void* stream)
{
    if (bytes == 0)
        return EVOSORT_OK;
    if (!dst || !src || (bytes & 3) || overlaps(dst, bytes, src, bytes))
        return EVOSORT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    EVOSORT_LAUNCH("stream_copy", s, launch_copy(dst, src, bytes, s));
    return EVOSORT_OK;
}

evosort_status evosort_stream_read(const void* src, size_t bytes, uint64_t* sink, void* stream)
{
    if (bytes == 0)
        return EVOSORT_OK;
    if (!src || !sink || (bytes & 15) || ((uintptr_t)src & 15))
        return EVOSORT_ERR_INVALID_ARG;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    EVOSORT_LAUNCH("stream_read", s, launch_stream_read(src, bytes, sink, s));
    return EVOSORT_OK;
}

void evosort_profile_enable(int on)
{
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = on != 0;
}

void evosort_profile_reset(void)
{
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto& r : P.pending) {
        P.pool.push_back(r.start);
        P.pool.push_back(r.stop);
    }
    P.pending.clear();
    P.totals.clear();
    P.names.clear();
}

int evosort_profile_collect(void)
{
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    for (auto& r : P.pending) {
        float ms = 0.f;
        if (hipEventSynchronize(r.stop) == hipSuccess && hipEventElapsedTime(&ms, r.start, r.stop) == hipSuccess) {
            auto it = P.totals.find(r.name);
            if (it == P.totals.end()) {
                P.names.push_back(r.name);
                P.totals[r.name] = {1, (double)ms};
            } else {
                it->second.first += 1;
                it->second.second += ms;
            }
        }
        P.pool.push_back(r.start);
        P.pool.push_back(r.stop);
    }
    P.pending.clear();
    return (int)P.names.size();
}

evosort_status evosort_profile_get(int i, char* name, size_t name_len, uint64_t* launches, double* total_ms)
{
    Profiler& P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (i < 0 || i >= (int)P.names.size())
        return EVOSORT_ERR_INVALID_ARG;
    const std::string& nm = P.names[i];
    if (name && name_len) {
        strncpy(name, nm.c_str(), name_len - 1);
        name[name_len - 1] = 0;
    }
    const auto& t = P.totals[nm];
    if (launches)
        *launches = t.first;
    if (total_ms)
        *total_ms = t.second;
    return EVOSORT_OK;
}

}  // extern "C"
