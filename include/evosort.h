/*
 * evosort.h -- C ABI of the EvoSort GPU sort library for AMD MI355X (gfx950).
 *
 * The library sorts one array of fixed-width keys on one GPU, ascending and
 * stably, optionally carrying one value per key, or returns the sorting
 * permutation.  It follows the paper's drop-in statement of the problem
 * (Sec. 1 and the opening of Sec. 4): one call takes an array and hands it
 * back sorted, usable wherever a library sort is; here the result is the one
 * a stable library sort gives.
 *
 * Two routines do the work and the adaptive partition sort chooses between
 * them (Sec. 4.3, Algorithm 6):
 *   - a block-based LSD radix sort (Sec. 4, Algorithms 4 and 5), built as an
 *     all-pass digit histogram, one device-wide scan of the digit counts and
 *     one single-sweep pass per digit with a decoupled look-back chained scan;
 *   - a bottom-up mergesort (Sec. 4, Algorithm 3): chunks of T_ins keys are
 *     sorted, then runs are merged pairwise with doubling length;
 *   - below a fallback threshold (the paper's T_numpy) one workgroup sorts the
 *     whole array (the paper hands such arrays to the platform's library sort).
 * The tunables of the paper's parameter vector (Sec. 3.2 and Sec. 4.2:
 * T_insertion, A_code, T_numpy) are fields of evosort_params, together with
 * the GPU's own knobs (digit width, tile shape).
 *
 * Key order.  Integer keys order by value.  Float keys order by IEEE-754
 * totalOrder: -NaN < -inf < ... < -0.0 < +0.0 < ... < +inf < +NaN.  Equal
 * keys keep their input order, so every routine and every parameter setting
 * gives the same bytes.
 *
 * Conventions for every call below:
 *   - Pointers named keys_*, vals_*, idx_*, temp, hist_*, bases_* are DEVICE
 *     pointers (hipMalloc'd or equivalent) on the current HIP device; sizes
 *     are element counts unless named *_bytes.  The caller owns all memory;
 *     the library never allocates device memory on a sort call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Work is enqueued on it and the call returns before the work ends; read
 *     the outputs after synchronizing that stream.
 *   - Argument errors are returned synchronously and nothing is enqueued.
 *     A failed HIP launch returns EVOSORT_ERR_HIP; evosort_last_hip_error()
 *     then gives the hipError_t of that failure (per host thread).
 *   - `temp` is scratch device memory of at least the size
 *     evosort_temp_bytes() reports for the same arguments; 256-byte alignment
 *     is required.  Its contents on entry do not matter.  Calls that share a
 *     temp buffer must not overlap in time.
 *   - In-place operation is allowed where stated (keys_out == keys_in,
 *     vals_out == vals_in).  Any other overlap between distinct input,
 *     output and temp buffers returns EVOSORT_ERR_INVALID_ARG.
 *   - All functions are safe to call from several host threads as long as
 *     their buffers are distinct.
 *   - Device-side errors.  A radix pass whose bounded look-back wait runs out
 *     (spin_limit) and a batch whose segment offsets break their rules fail
 *     after the call that enqueued them has returned.  Such a failure is
 *     recorded in that call's temp and in a host-visible word of the device,
 *     and reported once, by whichever comes first:
 *       - evosort_check_device_error on that call's temp (synchronizes);
 *       - the next evosort_sort, _sort_pairs, _argsort, _radix_pass,
 *         _segmented_sort(_pairs) or _sort_each call on the same device made
 *         after the failing kernel ran: it returns EVOSORT_ERR_DEVICE_TIMEOUT
 *         (EVOSORT_ERR_INVALID_ARG for bad offsets) and enqueues nothing.
 *     The outputs of the failed call are undefined.
 */
#ifndef EVOSORT_H_
#define EVOSORT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Key types. */
typedef enum evosort_dtype {
    EVOSORT_INT32 = 1,
    EVOSORT_INT64 = 2,
    EVOSORT_UINT32 = 3,
    EVOSORT_FLOAT32 = 4,
    EVOSORT_FLOAT64 = 5
} evosort_dtype;

/* Routine choice: the paper's A_code (Sec. 4.2): 3 = mergesort, 4 = LSD radix
 * sort.  0 = automatic: radix (the routine the paper's tuner picked at every
 * size, Sec. 6), except for keys-only sorts with no tile shape given whose key
 * type and length fall in a row of the GA tuner's table compiled into the
 * library (Sec. 4.2, Algorithm 2, run on an MI355X): there the row's routine,
 * the mergesort, is taken.  Other values are rejected with
 * EVOSORT_ERR_INVALID_ARG. */
typedef enum evosort_algo {
    EVOSORT_ALGO_AUTO = 0,
    EVOSORT_ALGO_MERGE = 3,
    EVOSORT_ALGO_RADIX = 4
} evosort_algo;

typedef enum evosort_status {
    EVOSORT_OK = 0,
    EVOSORT_ERR_INVALID_ARG = 1,       /* null pointer with n > 0, n < 0, bad overlap, bad param */
    EVOSORT_ERR_UNSUPPORTED_DTYPE = 2, /* dtype or value/index width not supported */
    EVOSORT_ERR_UNSUPPORTED_PARAM = 3, /* e.g. a tile shape that is not compiled in */
    EVOSORT_ERR_TEMP_TOO_SMALL = 4,    /* temp_bytes below evosort_temp_bytes() */
    EVOSORT_ERR_HIP = 5,               /* a HIP launch or runtime call failed */
    EVOSORT_ERR_DEVICE_TIMEOUT = 6,    /* a kernel's bounded wait ran out (see evosort_check_device_error) */
    EVOSORT_ERR_OVER_BUDGET = 7,       /* a served request needs more HBM than the server's whole budget */
    EVOSORT_ERR_PENDING = 8            /* a served request has not finished yet */
} evosort_status;

/* Operations, for evosort_temp_bytes and evosort_plan. */
typedef enum evosort_op {
    EVOSORT_OP_SORT = 0,       /* keys only */
    EVOSORT_OP_SORT_PAIRS = 1, /* keys and values of value_bytes each */
    EVOSORT_OP_ARGSORT = 2     /* keys in, permutation out, index of value_bytes (4 or 8) */
} evosort_op;

/* Routine a call takes (the branches of Sec. 4.3, Algorithm 6). */
typedef enum evosort_path {
    EVOSORT_PATH_COPY = 0,  /* n <= 1: at most a copy */
    EVOSORT_PATH_SMALL = 1, /* n below the fallback threshold: one workgroup sorts all */
    EVOSORT_PATH_RADIX = 2, /* block-based LSD radix sort */
    EVOSORT_PATH_MERGE = 3  /* bottom-up mergesort */
} evosort_path;

/* Debug switches (evosort_params.debug_flags).  Test use only. */
#define EVOSORT_DEBUG_WITHHOLD_TILE0 0x1u /* radix tile 0 never publishes its counts: later
                                            tiles run out of spin_limit and the call reports
                                            EVOSORT_ERR_DEVICE_TIMEOUT through the error word */
#define EVOSORT_DEBUG_WIDE_STATUS 0x2u    /* 64-bit look-back words at every n (normally only from
                                            n = 2^30 on), so that tests reach those kernels at
                                            small sizes; results are unchanged */

/*
 * Parameters.  Always initialise with evosort_default_params() and then change
 * fields; struct_size guards the ABI.
 *
 *   algo                 A_code: EVOSORT_ALGO_AUTO, _MERGE or _RADIX.
 *   digit_bits           radix digit width d, 4..12; the paper fixes 8 (Sec. 4,
 *                        Algorithms 4 and 5).  ceil(8*key_bytes/d) passes.
 *   insertion_threshold  T_ins, 1..2048 (the paper's bounds are [2, 2048],
 *                        Sec. 4.2): length of the chunks the mergesort sorts
 *                        before its first merge (Sec. 4, Algorithm 3).
 *   fallback_threshold   T_numpy: arrays with n < this go to the one-workgroup
 *                        sort.  Capped by what one workgroup holds
 *                        (evosort_plan reports the cap as small_capacity).
 *   block_threads,       GPU tile shape of the radix passes (threads per
 *   items_per_thread     workgroup, keys per thread); 0 = library default.
 *                        Only compiled-in shapes are accepted.
 *   spin_limit           bound on the look-back wait of a radix tile, in
 *                        polls; 0 = library default.  When it runs out the
 *                        kernel records EVOSORT_ERR_DEVICE_TIMEOUT in temp and
 *                        finishes (the output is then undefined).
 *   debug_flags          EVOSORT_DEBUG_* bits; 0 in normal use.
 *   descending           0: ascending order; 1: descending order, equal keys
 *                        still in input order (the order word is complemented;
 *                        floats: +NaN first, -0.0 after +0.0, -NaN last).
 */
typedef struct evosort_params {
    uint32_t struct_size;
    int32_t algo;
    uint32_t digit_bits;
    uint32_t insertion_threshold;
    uint64_t fallback_threshold;
    uint32_t block_threads;
    uint32_t items_per_thread;
    uint32_t spin_limit;
    uint32_t debug_flags;
    uint32_t descending;
    uint32_t reserved;
} evosort_params;

/* What a call with the given arguments would do (host only; no GPU needed). */
typedef struct evosort_plan_info {
    int32_t path;             /* evosort_path */
    uint32_t passes;          /* radix passes (0 unless path == RADIX) */
    uint32_t digit_bits;      /* effective d */
    uint32_t block_threads;   /* radix tile shape in effect */
    uint32_t items_per_thread;
    uint32_t status_bytes;    /* width of a look-back status word: 4 (n < 2^30) or 8 */
    uint64_t tile_keys;       /* keys per radix tile, or per mergesort block */
    uint64_t tiles;           /* radix tiles per pass, or mergesort blocks */
    uint32_t merge_rounds;    /* global merge rounds after the block sort (path == MERGE) */
    uint32_t reserved;
    uint64_t merge_block_run; /* sorted run length after the mergesort block sort */
    uint64_t small_capacity;  /* largest n the one-workgroup sort takes for this dtype/op */
    uint64_t temp_bytes;      /* same as evosort_temp_bytes */
} evosort_plan_info;

/* Fill *p with the defaults (struct_size set; algo AUTO; d = 8; T_ins = 8;
 * fallback = the one-workgroup capacity; default tile shape). */
void evosort_default_params(evosort_params *p);

/* Scratch size for an operation.  value_bytes: 0 for EVOSORT_OP_SORT, 4 or 8
 * otherwise (for ARGSORT it is the index width).  p may be NULL (defaults). */
evosort_status evosort_temp_bytes(int op, int dtype, int64_t n, uint32_t value_bytes,
                                  const evosort_params *p, size_t *out_bytes);

/* The routine and launch shape a call would use; host only. */
evosort_status evosort_plan(int op, int dtype, int64_t n, uint32_t value_bytes,
                            const evosort_params *p, evosort_plan_info *out);

/*
 * Sort keys (Sec. 4.3, Algorithm 6, and the routines it calls).
 * keys_in: n keys of `dtype`, read only unless keys_out == keys_in (in place).
 * keys_out: n keys, written with keys_in in ascending order (original bits).
 */
evosort_status evosort_sort(int dtype, const void *keys_in, void *keys_out, int64_t n, void *temp,
                            size_t temp_bytes, const evosort_params *p, void *stream);

/*
 * Sort key-value pairs stably by key.  Values are opaque value_bytes-wide
 * words (4 or 8) that travel with their keys; equal keys keep input order.
 * In place is allowed for keys and for values.
 */
evosort_status evosort_sort_pairs(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                  void *vals_out, uint32_t value_bytes, int64_t n, void *temp,
                                  size_t temp_bytes, const evosort_params *p, void *stream);

/*
 * Stable sorting permutation: idx_out[j] = input position of the key that a
 * stable sort places at j.  index_bytes 4 (int32, needs n <= 2^31 - 1) or 8
 * (int64).  keys_in is never written.
 */
evosort_status evosort_argsort(int dtype, const void *keys_in, void *idx_out, uint32_t index_bytes, int64_t n,
                               void *temp, size_t temp_bytes, const evosort_params *p, void *stream);

/*
 * Allocation-free sort, for callers that cannot allocate device memory or
 * call allocating routines (code under HIP graph capture, tight serving
 * loops, harnesses that forbid it).  The same sort as evosort_sort, with its
 * scratch in a device array inside the library instead of a caller's temp:
 * EVOSORT_NOALLOC_SCRATCH_BYTES per device, held from the library's load on
 * that device until the process ends.  The call allocates, creates and frees
 * nothing (profiling events are not recorded for it).
 *   - Sizes whose scratch (evosort_plan(EVOSORT_OP_SORT, ...).temp_bytes of
 *     the routine the call takes) exceeds EVOSORT_NOALLOC_SCRATCH_BYTES return
 *     EVOSORT_ERR_TEMP_TOO_SMALL and enqueue nothing (about 16e6 4-byte or
 *     8e6 8-byte keys fit).
 *   - Every call on a device shares that device's array, which keeps the last
 *     call's contents; each call clears what must start at zero.  Calls that
 *     overlap in time on one device (other streams, other host threads) race
 *     on the array and give undefined results: serialize them.
 *   - Device-side errors are reported at the next call as for evosort_sort;
 *     evosort_check_device_error does not apply (there is no temp).
 */
#define EVOSORT_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
evosort_status evosort_sort_noalloc(int dtype, const void *keys_in, void *keys_out, int64_t n,
                                    const evosort_params *p, void *stream);

/* ------------------------------------------------------------------------ */
/* Single steps of the two routines, exported so each can be checked alone.  */
/* ------------------------------------------------------------------------ */

/*
 * Radix steps 1-2: digit histograms of all passes and their exclusive prefix
 * sums (Sec. 4, Algorithm 4: per-thread counts combined into one histogram
 * per pass, then prefix sums; here one read of the keys serves every pass).
 * hist_out and bases_out: device arrays of passes * 2^digit_bits uint64,
 * row p = pass p (digit bits [p*d, p*d + d) of the order key).  bases_out may
 * be NULL.  temp as for evosort_sort with the same dtype and n.
 */
evosort_status evosort_radix_histogram(int dtype, const void *keys, int64_t n, uint32_t digit_bits,
                                       uint64_t *hist_out, uint64_t *bases_out, void *temp, size_t temp_bytes,
                                       void *stream);

/*
 * Radix step 3: one stable LSD pass on digit `pass` (Sec. 4, Algorithm 4,
 * loop body: offsets, then placement into the other buffer).  Equivalent to a
 * stable counting sort of the input on that digit.  vals may be NULL
 * (value_bytes 0).  Not in place.  temp as for evosort_sort_pairs (or
 * evosort_sort when keys only) with the same arguments.
 */
evosort_status evosort_radix_pass(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                  void *vals_out, uint32_t value_bytes, int64_t n, uint32_t pass,
                                  void *temp, size_t temp_bytes, const evosort_params *p, void *stream);

/*
 * Mergesort step 1: sort every block of the mergesort on its own: each block
 * of evosort_plan().merge_block_run keys is cut into chunks of T_ins keys,
 * each chunk is sorted, then the chunks are merged pairwise inside the block
 * (Sec. 4, Algorithm 3, first loop and the first merge rounds).  Not in place.
 * *run_out receives the run length produced.
 */
evosort_status evosort_merge_block_sort(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                        void *vals_out, uint32_t value_bytes, int64_t n, const evosort_params *p,
                                        int64_t *run_out, void *stream);

/*
 * Mergesort step 2: one merge round (Sec. 4, Algorithm 3, while-loop body):
 * runs [2k*run, (2k+1)*run) and [(2k+1)*run, (2k+2)*run) of keys_in, each
 * sorted, are merged into keys_out (ties take the left run; a trailing run
 * without a partner is copied).  Not in place.  temp: the merge-path split
 * points of this round; 256 + 8 * (n + 4) bytes always suffice
 * (EVOSORT_ERR_TEMP_TOO_SMALL otherwise).
 */
evosort_status evosort_merge_round(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                   void *vals_out, uint32_t value_bytes, int64_t n, int64_t run, void *temp,
                                   size_t temp_bytes, void *stream);

/* ------------------------------------------------------------------------ */
/* Batches of arrays.                                                        */
/* ------------------------------------------------------------------------ */

/*
 * Batched segmented sort.  Segment i is keys [offsets[i], offsets[i+1]) and is
 * sorted on its own, ascending and stably: the result equals evosort_sort
 * (evosort_sort_pairs) applied to each segment alone.
 *
 *   offsets    DEVICE array of nseg + 1 int64, non-decreasing, within [0, n],
 *              every segment shorter than 2^30 keys.  Keys outside
 *              [offsets[0], offsets[nseg]) are neither read nor written.
 *              The offsets are checked on the device before anything else:
 *              if any breaks these rules, no key or value is written and
 *              evosort_check_device_error() returns EVOSORT_ERR_INVALID_ARG.
 *   size classes  a segment shorter than fallback_threshold that fits one
 *              workgroup (evosort_segmented_capacity) is sorted by one
 *              workgroup in LDS (the small-array branch of Sec. 4.3,
 *              Algorithm 6, per segment); longer segments take the
 *              single-sweep LSD passes (Sec. 4, Algorithms 4 and 5), each
 *              segment with its own digit histogram and chained scan.
 *   params     digit_bits must be 8 and algo AUTO or RADIX
 *              (EVOSORT_ERR_UNSUPPORTED_PARAM otherwise); block_threads and
 *              items_per_thread pick the tile shape of the long segments.
 *   graphs     the call is one fixed sequence of kernel launches: every
 *              decision that depends on the segment sizes is taken on the
 *              GPU, and nothing is allocated, synchronized or memset, so the
 *              call can be captured in a HIP graph; a replay reads the
 *              offsets, keys and values present at replay time.
 *   temp       evosort_segmented_temp_bytes(dtype, n, nseg, value_bytes, p).
 * In place is allowed for keys and for values.
 */
evosort_status evosort_segmented_temp_bytes(int dtype, int64_t n, int64_t nseg, uint32_t value_bytes,
                                            const evosort_params *p, size_t *out_bytes);
evosort_status evosort_segmented_sort(int dtype, const void *keys_in, void *keys_out, int64_t n,
                                      const int64_t *offsets, int64_t nseg, void *temp, size_t temp_bytes,
                                      const evosort_params *p, void *stream);
evosort_status evosort_segmented_sort_pairs(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                            void *vals_out, uint32_t value_bytes, int64_t n,
                                            const int64_t *offsets, int64_t nseg, void *temp, size_t temp_bytes,
                                            const evosort_params *p, void *stream);

/* Largest segment the one-workgroup classes take for (dtype, value_bytes). */
evosort_status evosort_segmented_capacity(int dtype, uint32_t value_bytes, int64_t *out_keys);

/*
 * Synchronize `stream` and read what the last segmented call on `temp` did:
 * class_counts[0..3] = segments per one-workgroup class (smallest first;
 * unused classes 0), class_counts[4] = segments that took the radix passes;
 * *tiles = radix tiles per pass.  Either output may be NULL.
 */
evosort_status evosort_segmented_stats(const void *temp, size_t temp_bytes, uint32_t *class_counts,
                                       uint32_t *tiles, void *stream);

/*
 * The same batch sorted one segment at a time: one evosort_sort (values
 * NULL, value_bytes 0) or evosort_sort_pairs per non-empty segment, in order,
 * on `stream` -- the schedule the segmented sort replaces.  host_offsets is a
 * HOST array of nseg + 1 int64 with the rules above.  temp as
 * evosort_temp_bytes for the longest segment.
 */
evosort_status evosort_sort_each(int dtype, const void *keys_in, void *keys_out, const void *vals_in,
                                 void *vals_out, uint32_t value_bytes, const int64_t *host_offsets, int64_t nseg,
                                 void *temp, size_t temp_bytes, const evosort_params *p, void *stream);

/* ------------------------------------------------------------------------ */
/* Serving: a request loop with continuous batching.                          */
/* ------------------------------------------------------------------------ */

/*
 * A sort server admits sort requests of any length and key type and runs
 * them on one GPU while others are still arriving (the paper's adaptive,
 * drop-in sort offered as a service; Sec. 1 and Sec. 4.3).  It owns one
 * device arena of hbm_budget_bytes, reserved once at creation: every admitted
 * request's output and scratch come from it, so the budget bounds the HBM the
 * server holds at any time.  A scheduler thread:
 *   - admits waiting requests in arrival order (first in, first out) while a
 *     stream slot is free and the arena can hold the request's output and
 *     scratch; a request that does not fit waits for releases (no request
 *     overtakes an earlier one);
 *   - packs consecutive waiting requests of one key type that are at most
 *     batch_max_keys long into one batch: their keys are gathered into one
 *     arena buffer and sorted by one batched segmented sort, in place;
 *   - runs each longer request as its own evosort_sort call;
 *   - runs up to `streams` jobs (batches or single requests) at once, each on
 *     its own HIP stream, so work admitted at different times overlaps on
 *     the device, and retires jobs as their streams finish.
 * Every result is the one evosort_sort gives for that request alone: the
 * stable sort is unique, whatever the batch or the other work on the GPU.
 *
 * Results stay in the arena (device-resident) until evosort_server_release;
 * a client that never releases stalls admission once the arena is full.
 */
typedef struct evosort_server evosort_server;

typedef struct evosort_server_config {
    uint32_t struct_size;      /* set by evosort_server_default_config */
    uint32_t streams;          /* concurrent jobs (HIP streams), 1..16; default 4 */
    uint64_t hbm_budget_bytes; /* arena size in bytes; default 1 GiB */
    uint64_t batch_max_keys;   /* requests of at most this many keys are batched; 0 = no batching;
                                  default 65536 */
    uint32_t batch_max_requests; /* requests per batch, 1..8192; default 2048 */
    uint32_t reserved;
    evosort_params params;     /* parameters of every sort the server runs (default params) */
} evosort_server_config;

typedef struct evosort_server_stats {
    uint64_t submitted, completed, released, failed;
    uint64_t jobs;             /* batches and single requests launched */
    uint64_t batched_requests; /* requests that ran inside a batch */
    uint64_t keys_completed;
    uint64_t bytes_in_use;     /* arena bytes held now (running and unreleased results) */
    uint64_t peak_bytes;       /* most arena bytes held at once */
    uint64_t budget_bytes;
    uint32_t max_concurrent_jobs; /* most jobs on the GPU at once */
    uint32_t waiting;          /* requests not yet admitted */
} evosort_server_stats;

void evosort_server_default_config(evosort_server_config *cfg);

/* Create a server on the current HIP device.  Reserves the arena (the only
 * device allocation the server makes), the streams and pinned staging. */
evosort_status evosort_server_create(const evosort_server_config *cfg, evosort_server **out);

/* Wait for every admitted request, stop the scheduler and free everything.
 * Results not yet copied out are lost.  Requests still waiting are dropped. */
evosort_status evosort_server_destroy(evosort_server *srv);

/*
 * Submit a request: n keys of `dtype` at DEVICE pointer keys_in, which must
 * stay valid and unchanged until the request completes (it is only read).
 * Returns at once with *id.  EVOSORT_ERR_OVER_BUDGET if the request could
 * never fit in the arena.
 */
evosort_status evosort_server_submit(evosort_server *srv, int dtype, const void *keys_in, int64_t n, uint64_t *id);

/* Non-blocking: EVOSORT_OK and *keys_out (DEVICE pointer into the arena,
 * valid until release) once done; EVOSORT_ERR_PENDING while not; the sort's
 * error status if it failed. */
evosort_status evosort_server_result(evosort_server *srv, uint64_t id, const void **keys_out);

/* Block until request id is done; then as evosort_server_result. */
evosort_status evosort_server_wait(evosort_server *srv, uint64_t id, const void **keys_out);

/* Copy a finished result to dst (DEVICE pointer, n keys) on `stream`. */
evosort_status evosort_server_copy_out(evosort_server *srv, uint64_t id, void *dst, void *stream);

/* Host times of a finished request, in milliseconds since the server was
 * created: submitted, admitted (launched), finished (its stream observed
 * done by the scheduler, which polls every few microseconds while busy). */
evosort_status evosort_server_times(evosort_server *srv, uint64_t id, double *submit_ms, double *admit_ms,
                                    double *done_ms);

/* Give a finished request's arena memory back (its result pointer dies). */
evosort_status evosort_server_release(evosort_server *srv, uint64_t id);

/* Block until every submitted request is done. */
evosort_status evosort_server_drain(evosort_server *srv);

evosort_status evosort_server_get_stats(evosort_server *srv, evosort_server_stats *out);

/* ------------------------------------------------------------------------ */
/* Errors and measurement.                                                   */
/* ------------------------------------------------------------------------ */

/* Static text for a status code. */
const char *evosort_status_string(int status);

/* hipError_t behind the last EVOSORT_ERR_HIP on this host thread (0 if none). */
int evosort_last_hip_error(void);

/* Identity of the built library: the first 16 hex digits of the SHA-256 of
 * its source files (every file of the package's csrc/ directory and of
 * include/, in name order, each as its relative path, a NUL byte and its
 * bytes), fixed when the library was compiled.  Static string. */
const char *evosort_build_id(void);

/*
 * Synchronize `stream` and read the device error word a sort or segmented
 * call left in `temp`: EVOSORT_OK, EVOSORT_ERR_DEVICE_TIMEOUT if a look-back
 * wait ran out of spin_limit, or EVOSORT_ERR_INVALID_ARG if segment offsets
 * broke their rules.  temp/temp_bytes as passed to that call (every routine
 * clears the word when it starts, so a temp reused by a later call reports
 * that call).  An error found here is not reported again by the next call.
 */
evosort_status evosort_check_device_error(const void *temp, size_t temp_bytes, void *stream);

/*
 * Streaming kernels that bound the sort kernels from above, for measuring
 * them (the roofline every radix pass and histogram is compared against):
 *   evosort_stream_copy  reads and writes every byte once (16-byte accesses,
 *                        a grid-stride loop), like one radix pass; `bytes` a
 *                        multiple of 4; the library's own device-to-device
 *                        copies use the same kernel.  dst and src must not
 *                        overlap (EVOSORT_ERR_INVALID_ARG).
 *   evosort_stream_read  reads every byte once and writes (almost) nothing,
 *                        like the all-pass histogram; `bytes` a multiple of
 *                        16, src 16-byte aligned; `sink` is one device word it
 *                        may write.
 * Both are enqueued on `stream` like the sorts.
 */
evosort_status evosort_stream_copy(void *dst, const void *src, size_t bytes, void *stream);
evosort_status evosort_stream_read(const void *src, size_t bytes, uint64_t *sink, void *stream);

/*
 * Kernel timing with HIP events.  While enabled, every kernel launch of the
 * library is bracketed by two events recorded on the launch stream.
 * evosort_profile_collect synchronizes those events and folds them into
 * per-kernel totals; evosort_profile_get reads kernel i (0 <= i < count).
 * Off by default; costs two event records per launch when on.
 */
void evosort_profile_enable(int on);
void evosort_profile_reset(void);
int evosort_profile_collect(void);
evosort_status evosort_profile_get(int i, char *name, size_t name_len, uint64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* EVOSORT_H_ */
