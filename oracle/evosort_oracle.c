/*
 * evosort_oracle.c -- reference oracle for the EvoSort sort path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is compiled into liboracle.so, which
 * only the test-suite, the package smoke check and the benchmark's CPU-baseline
 * leg load.  The GPU library never links, loads or calls it, and it includes no
 * header of the GPU library: it carries its own key-order function and its own
 * kind codes.
 *
 * What it computes.  Sorting reaches a result with a plain definition, so the
 * oracle writes that definition out:
 *
 *   u[i]  = the order key of keys[i] (an unsigned integer whose natural order
 *           is the order of the key type; see order_key below),
 *   perm  = the unique stable sorting permutation: indices ordered by u
 *           ascending, equal u ordered by index ascending,
 *   out[j]= keys[perm[j]]   (values and argsort follow from perm).
 *
 * The descending sort is the same definition with u ordered descending (equal
 * u still by index ascending): the stable sort a caller asking for
 * descending order expects.
 *
 * perm is computed by a textbook top-down stable mergesort (ties take the left
 * run), single-threaded.  Besides the whole sort, the file holds the single
 * steps the paper's two sort routines are built from, each written from the
 * paper's description, so that the GPU steps can be checked one at a time:
 *
 *   - oracle_digit_histogram : per-digit counts of every radix pass
 *                              (Sec. 4, Algorithm 4, RefinedParallelRadixSort_int32,
 *                              histogram step; 8-bit digits there, width free here)
 *   - oracle_counting_pass   : one stable LSD pass on one digit (same algorithm,
 *                              prefix-sum + scatter step)
 *   - oracle_insertion_chunks: insertion sort of every chunk of a given length
 *                              (Sec. 4, Algorithm 3, RefinedParallelMergeSort, first loop)
 *   - oracle_merge_round     : one merge round over pairs of adjacent sorted runs
 *                              (same algorithm, while-loop body)
 *   - oracle_rank_of         : the output position of one input element under
 *                              the stable sort, by counting (for sampled checks
 *                              at sizes the full sort is too slow for)
 *
 * Readings of the paper used here (the paper is silent on them):
 *   - floating-point keys order by IEEE-754 totalOrder (-0.0 before +0.0,
 *     negative-signed NaNs first, positive NaNs last); the paper sorts only
 *     integers with its radix routine;
 *   - equal keys keep their input order (stability); the paper's check is on
 *     plain integers, where stability is invisible;
 *   - a merge round leaves a trailing run without a partner unchanged.
 *
 * All functions return 0 on success and a negative value on a bad argument.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Key kinds understood by the oracle (its own numbering). */
enum {
    ORK_INT32 = 1,
    ORK_INT64 = 2,
    ORK_UINT32 = 3,
    ORK_FLOAT32 = 4,
    ORK_FLOAT64 = 5
};

static int kind_bytes(int kind)
{
    switch (kind) {
    case ORK_INT32:
    case ORK_UINT32:
    case ORK_FLOAT32:
        return 4;
    case ORK_INT64:
    case ORK_FLOAT64:
        return 8;
    default:
        return 0;
    }
}

/*
 * Order key: an unsigned integer u with  a < b  in the key type's order
 * exactly when u(a) < u(b).
 *
 *  - signed integers: offset binary, u = v - INT_MIN, computed as an integer
 *    addition (the paper flips the sign bit with XOR 0x80000000 and
 *    0x8000000000000000, Sec. 4, Algorithms 4 and 5; for two's complement this is the same map);
 *  - unsigned 32-bit: u = v;
 *  - IEEE floats: a value with the sign bit set is negative (or -0.0 or a
 *    negative-signed NaN): larger magnitude must give a smaller key, so the
 *    key is the bitwise complement of the pattern; a value with the sign bit
 *    clear gets the sign bit set, placing it above every negative one.
 */
static uint64_t order_key(int kind, const unsigned char *base, int64_t i)
{
    switch (kind) {
    case ORK_INT32: {
        int32_t v;
        memcpy(&v, base + 4 * i, 4);
        return (uint64_t)((int64_t)v + 2147483648LL);
    }
    case ORK_UINT32: {
        uint32_t v;
        memcpy(&v, base + 4 * i, 4);
        return (uint64_t)v;
    }
    case ORK_INT64: {
        int64_t v;
        memcpy(&v, base + 8 * i, 8);
        /* (uint64)v is v mod 2^64; adding 2^63 mod 2^64 gives v + 2^63. */
        return (uint64_t)v + (UINT64_C(1) << 63);
    }
    case ORK_FLOAT32: {
        uint32_t b;
        memcpy(&b, base + 4 * i, 4);
        if (b & 0x80000000u)
            return (uint64_t)(uint32_t)~b;
        return (uint64_t)(b | 0x80000000u);
    }
    case ORK_FLOAT64: {
        uint64_t b;
        memcpy(&b, base + 8 * i, 8);
        if (b & (UINT64_C(1) << 63))
            return ~b;
        return b | (UINT64_C(1) << 63);
    }
    default:
        return 0;
    }
}

/* Exported so that tests can check the key order directly. */
int oracle_order_keys(int kind, const void *keys, int64_t n, uint64_t *u_out)
{
    if (!kind_bytes(kind) || n < 0 || (n > 0 && (!keys || !u_out)))
        return -1;
    for (int64_t i = 0; i < n; ++i)
        u_out[i] = order_key(kind, (const unsigned char *)keys, i);
    return 0;
}

typedef struct {
    uint64_t u;  /* order key */
    int64_t idx; /* input position */
} record_t;

static record_t *make_records(int kind, const void *keys, int64_t n)
{
    record_t *r = (record_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(record_t));
    if (!r)
        return NULL;
    for (int64_t i = 0; i < n; ++i) {
        r[i].u = order_key(kind, (const unsigned char *)keys, i);
        r[i].idx = i;
    }
    return r;
}

/* Textbook top-down mergesort of r[lo, hi) using tmp as the merge buffer.
 * Ascending: the merge takes from the left half unless the right element is
 * strictly smaller; descending: unless it is strictly larger.  Either way
 * equal keys keep their order. */
static void mergesort_records(record_t *r, record_t *tmp, int64_t lo, int64_t hi, int descending)
{
    if (hi - lo < 2)
        return;
    int64_t mid = lo + (hi - lo) / 2;
    mergesort_records(r, tmp, lo, mid, descending);
    mergesort_records(r, tmp, mid, hi, descending);
    int64_t a = lo, b = mid, k = lo;
    while (a < mid && b < hi) {
        const int right_first = descending ? (r[b].u > r[a].u) : (r[b].u < r[a].u);
        if (right_first)
            tmp[k++] = r[b++];
        else
            tmp[k++] = r[a++];
    }
    while (a < mid)
        tmp[k++] = r[a++];
    while (b < hi)
        tmp[k++] = r[b++];
    memcpy(r + lo, tmp + lo, (size_t)(hi - lo) * sizeof(record_t));
}

/* The stable sorting permutation of keys[0, n), ascending (descending = 0)
 * or descending (descending = 1): indices ordered by the order key in that
 * direction, equal keys by index ascending in both. */
int oracle_stable_perm_dir(int kind, const void *keys, int64_t n, int descending, int64_t *perm_out)
{
    if (!kind_bytes(kind) || n < 0 || (n > 0 && (!keys || !perm_out)))
        return -1;
    if (n == 0)
        return 0;
    record_t *r = make_records(kind, keys, n);
    record_t *tmp = (record_t *)malloc((size_t)n * sizeof(record_t));
    if (!r || !tmp) {
        free(r);
        free(tmp);
        return -2;
    }
    mergesort_records(r, tmp, 0, n, descending ? 1 : 0);
    for (int64_t j = 0; j < n; ++j)
        perm_out[j] = r[j].idx;
    free(r);
    free(tmp);
    return 0;
}

/* The ascending stable sorting permutation of keys[0, n). */
int oracle_stable_perm(int kind, const void *keys, int64_t n, int64_t *perm_out)
{
    return oracle_stable_perm_dir(kind, keys, n, 0, perm_out);
}

/* Number of digit positions needed to cover a key of kbytes bytes. */
static int pass_count(int kbytes, int digit_bits)
{
    return (8 * kbytes + digit_bits - 1) / digit_bits;
}

/*
 * Digit histograms of all passes: hist[p * 2^bits + d] = number of keys whose
 * digit p (bits [p*bits, p*bits + bits) of the order key) equals d.  The last
 * digit of a key whose width is not a multiple of bits is narrower; its high
 * bins stay zero.
 */
int oracle_digit_histogram(int kind, const void *keys, int64_t n, int digit_bits, uint64_t *hist)
{
    int kb = kind_bytes(kind);
    if (!kb || n < 0 || digit_bits < 1 || digit_bits > 16 || !hist || (n > 0 && !keys))
        return -1;
    int passes = pass_count(kb, digit_bits);
    uint64_t bins = UINT64_C(1) << digit_bits;
    memset(hist, 0, (size_t)passes * bins * sizeof(uint64_t));
    for (int64_t i = 0; i < n; ++i) {
        uint64_t u = order_key(kind, (const unsigned char *)keys, i);
        for (int p = 0; p < passes; ++p) {
            int shift = p * digit_bits;
            uint64_t d = (u >> shift) & (bins - 1);
            hist[(uint64_t)p * bins + d] += 1;
        }
    }
    return 0;
}

/*
 * One stable counting pass on the digit at bit offset `shift`: count the keys
 * per digit, turn the counts into exclusive prefix sums (the first output
 * position of each digit), then place the keys in input order.  perm_out[j]
 * is the input position of the key placed at output position j.
 */
int oracle_counting_pass(int kind, const void *keys, int64_t n, int shift, int digit_bits,
                         int64_t *perm_out)
{
    int kb = kind_bytes(kind);
    if (!kb || n < 0 || digit_bits < 1 || digit_bits > 16 || shift < 0 || shift >= 8 * kb ||
        (n > 0 && (!keys || !perm_out)))
        return -1;
    uint64_t bins = UINT64_C(1) << digit_bits;
    uint64_t *next = (uint64_t *)calloc((size_t)bins, sizeof(uint64_t));
    if (!next)
        return -2;
    for (int64_t i = 0; i < n; ++i) {
        uint64_t u = order_key(kind, (const unsigned char *)keys, i);
        next[(u >> shift) & (bins - 1)] += 1;
    }
    uint64_t run = 0;
    for (uint64_t d = 0; d < bins; ++d) {
        uint64_t c = next[d];
        next[d] = run;
        run += c;
    }
    for (int64_t i = 0; i < n; ++i) {
        uint64_t u = order_key(kind, (const unsigned char *)keys, i);
        uint64_t d = (u >> shift) & (bins - 1);
        perm_out[next[d]++] = i;
    }
    free(next);
    return 0;
}

/*
 * Insertion sort of each chunk [c*chunk, min((c+1)*chunk, n)) on its own.
 * The inner loop moves an element left past strictly greater keys only, so
 * equal keys keep their order.
 */
int oracle_insertion_chunks(int kind, const void *keys, int64_t n, int64_t chunk, int64_t *perm_out)
{
    if (!kind_bytes(kind) || n < 0 || chunk < 1 || (n > 0 && (!keys || !perm_out)))
        return -1;
    if (n == 0)
        return 0;
    record_t *r = make_records(kind, keys, n);
    if (!r)
        return -2;
    for (int64_t lo = 0; lo < n; lo += chunk) {
        int64_t hi = lo + chunk < n ? lo + chunk : n;
        for (int64_t i = lo + 1; i < hi; ++i) {
            record_t x = r[i];
            int64_t j = i - 1;
            while (j >= lo && r[j].u > x.u) {
                r[j + 1] = r[j];
                --j;
            }
            r[j + 1] = x;
        }
    }
    for (int64_t j = 0; j < n; ++j)
        perm_out[j] = r[j].idx;
    free(r);
    return 0;
}

/*
 * One merge round: runs [2k*run, (2k+1)*run) and [(2k+1)*run, (2k+2)*run)
 * (clipped to n) are each assumed sorted and are merged into one run; a tie
 * takes the element of the left run.  A last run without a partner is copied
 * unchanged.
 */
int oracle_merge_round(int kind, const void *keys, int64_t n, int64_t run, int64_t *perm_out)
{
    if (!kind_bytes(kind) || n < 0 || run < 1 || (n > 0 && (!keys || !perm_out)))
        return -1;
    if (n == 0)
        return 0;
    record_t *r = make_records(kind, keys, n);
    if (!r)
        return -2;
    int64_t k = 0;
    for (int64_t lo = 0; lo < n; lo += 2 * run) {
        int64_t mid = lo + run < n ? lo + run : n;
        int64_t hi = lo + 2 * run < n ? lo + 2 * run : n;
        int64_t a = lo, b = mid;
        while (a < mid && b < hi) {
            if (r[b].u < r[a].u)
                perm_out[k++] = r[b++].idx;
            else
                perm_out[k++] = r[a++].idx;
        }
        while (a < mid)
            perm_out[k++] = r[a++].idx;
        while (b < hi)
            perm_out[k++] = r[b++].idx;
    }
    free(r);
    return 0;
}

/*
 * Output position of input element i under the stable sort:
 *   #{k : u[k] < u[i]} + #{k < i : u[k] == u[i]}.
 * One pass over the keys; used to check sampled outputs of large sorts.
 */
int oracle_rank_of(int kind, const void *keys, int64_t n, int64_t i, int64_t *rank_out)
{
    if (!kind_bytes(kind) || n < 0 || i < 0 || i >= n || !keys || !rank_out)
        return -1;
    const unsigned char *base = (const unsigned char *)keys;
    uint64_t ui = order_key(kind, base, i);
    int64_t rank = 0;
    for (int64_t k = 0; k < n; ++k) {
        uint64_t uk = order_key(kind, base, k);
        if (uk < ui || (uk == ui && k < i))
            ++rank;
    }
    *rank_out = rank;
    return 0;
}

/*
 * Property check for outputs too large to sort on the host: returns the first
 * j with u[j] > u[j+1], or -1 if keys[0, n) is in non-decreasing order.
 */
int64_t oracle_first_unsorted(int kind, const void *keys, int64_t n)
{
    if (!kind_bytes(kind) || n < 0 || (n > 0 && !keys))
        return -2;
    const unsigned char *base = (const unsigned char *)keys;
    for (int64_t j = 0; j + 1 < n; ++j)
        if (order_key(kind, base, j) > order_key(kind, base, j + 1))
            return j;
    return -1;
}
