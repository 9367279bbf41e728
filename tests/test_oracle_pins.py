"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test ties one oracle function to something fixed independently of it:
values the paper fixes (the sign-flip masks, the pass counts, the dispatch
branches), a published ordering standard (IEEE-754 totalOrder), a library
routine that solves a special case (numpy's stable sort on integers, Python's
stable ``sorted``), brute force over every input of a tiny alphabet, or an
invariant that any correct sort satisfies.  None of these call the GPU library.
"""
import itertools
import math
import struct

import numpy as np
import pytest

import oracle
import workloads
from conftest import read_golden

INT_DTYPES = [np.int32, np.int64, np.uint32]
ALL_DTYPES = [np.int32, np.int64, np.uint32, np.float32, np.float64]


# --------------------------------------------------------------------------
# Key order
# --------------------------------------------------------------------------
def test_sign_flip_matches_paper_masks():
    """Signed keys: order key = value XOR sign mask (masks of Sec. 4, Algorithms 4 and 5), from a golden table."""
    rows = read_golden("int_sign_flip.txt")
    assert rows
    for dt, val, mapped in rows:
        a = np.array([int(val)], dtype=np.dtype(dt))
        assert int(oracle.order_keys(a)[0]) == int(mapped, 16), (dt, val)


@pytest.mark.parametrize("dt", ["float32", "float64"])
def test_float_order_is_ieee_total_order(dt):
    rows = [r for r in read_golden("float_total_order.txt") if r[0] == dt]
    assert len(rows) == 16
    bits = np.array([int(r[1], 16) for r in rows], dtype=np.uint32 if dt == "float32" else np.uint64)
    vals = bits.view(np.dtype(dt))
    u = oracle.order_keys(vals)
    assert np.all(np.diff(u.astype(object)) > 0), "golden rows must map to strictly ascending keys"
    # any permutation of the rows sorts back to the golden order
    g = np.random.default_rng(3)
    for _ in range(20):
        p = g.permutation(len(vals))
        got = oracle.sort(vals[p]).view(bits.dtype)
        assert np.array_equal(got, bits)


def test_uint32_key_is_identity():
    x = workloads.uniform(np.uint32, 1000, 5)
    assert np.array_equal(oracle.order_keys(x), x.astype(np.uint64))


def test_int_order_key_monotone_on_random_pairs():
    for dt in (np.int32, np.int64):
        x = workloads.uniform(dt, 20000, 11)
        u = oracle.order_keys(x)
        a, b = x[:-1].astype(object), x[1:].astype(object)
        ua, ub = u[:-1].astype(object), u[1:].astype(object)
        for i in range(len(a)):
            assert (a[i] < b[i]) == (ua[i] < ub[i])
            assert (a[i] == b[i]) == (ua[i] == ub[i])


# --------------------------------------------------------------------------
# Whole sort: brute force on tiny inputs
# --------------------------------------------------------------------------
def _selection_perm(vals, key):
    """O(n^2) selection of the smallest (key, index) pair, written apart from the oracle."""
    left = list(range(len(vals)))
    out = []
    while left:
        best = left[0]
        for i in left[1:]:
            if (key(vals[i]), i) < (key(vals[best]), best):
                best = i
        out.append(best)
        left.remove(best)
    return out


@pytest.mark.parametrize("dt,alphabet", [
    (np.int32, [-2, -1, 0, 1, 2]),
    (np.int64, [-(2**63), -1, 0, 1, 2**63 - 1]),
    (np.uint32, [0, 1, 2, 2**31, 2**32 - 1]),
])
def test_brute_force_all_small_integer_inputs(dt, alphabet):
    for length in range(0, 7):
        for combo in itertools.product(alphabet, repeat=length):
            keys = np.array(combo, dtype=dt)
            expect = _selection_perm(list(combo), key=lambda v: v)
            assert oracle.stable_perm(keys).tolist() == expect, combo


def _float_key(v):
    # value first; -0.0 and +0.0 compare equal as numbers, the sign decides between them
    return (v, math.copysign(1.0, v))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_brute_force_all_small_float_inputs(dt):
    alphabet = [-math.inf, -1.5, -0.0, 0.0, 1.5, math.inf]
    for length in range(0, 6):
        for combo in itertools.product(alphabet, repeat=length):
            keys = np.array(combo, dtype=dt)
            expect = _selection_perm(list(combo), key=_float_key)
            assert oracle.stable_perm(keys).tolist() == expect, combo


# --------------------------------------------------------------------------
# Whole sort: library special cases and invariants
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dt", INT_DTYPES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 100, 4097, 100_003])
def test_integer_sort_equals_numpy_stable(dt, n):
    g = np.random.default_rng(n + 17)
    for keys in (workloads.uniform(dt, n, n), g.integers(0, 7, size=n).astype(dt)):
        perm = oracle.stable_perm(keys)
        assert np.array_equal(perm, np.argsort(keys, kind="stable"))
        assert np.array_equal(oracle.sort(keys), np.sort(keys, kind="stable"))


@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_float_sort_equals_numpy_without_signed_zero_or_nan(dt):
    x = workloads.gaussian(dt, 50_000, 9, sd=3.0)
    x[::97] = np.inf
    x[::89] = -np.inf
    x[x == 0] = 1.0  # numpy treats -0.0 == +0.0; keep the special case clean
    assert np.array_equal(oracle.stable_perm(x), np.argsort(x, kind="stable"))


@pytest.mark.parametrize("dt", ALL_DTYPES)
@pytest.mark.parametrize("dist", ["uniform", "distinct16", "all_equal"])
def test_sort_invariants(dt, dist):
    n = 30_011
    keys = workloads.make(dist, dt, n, 21) if dist != "uniform" else workloads.uniform(dt, n, 21)
    perm = oracle.stable_perm(keys)
    # a permutation
    assert np.array_equal(np.sort(perm), np.arange(n))
    out = keys[perm]
    # ordered (checked with Python comparisons on the total-order keys of the golden table)
    u = oracle.order_keys(out)
    assert np.all(u[:-1] <= u[1:])
    # same multiset of bit patterns
    bits = {4: np.uint32, 8: np.uint64}[keys.dtype.itemsize]
    assert np.array_equal(np.sort(out.view(bits)), np.sort(keys.view(bits)))
    # stable: equal keys keep increasing input positions
    same = u[:-1] == u[1:]
    assert np.all(perm[:-1][same] < perm[1:][same])


def test_float_mix_places_signed_zeros_and_infinities():
    x = workloads.float_mix(np.float64, 20_000, 4, frac=0.05)
    out = oracle.sort(x)
    assert np.isneginf(out[0]) and np.isposinf(out[-1])
    z = np.flatnonzero(out == 0)
    signs = np.signbit(out[z])
    # all -0.0 come before all +0.0, and the zero block is contiguous
    assert np.all(np.diff(z) == 1)
    assert not np.any(signs[1:] & ~signs[:-1])


def test_pairs_and_argsort_follow_the_permutation():
    g = np.random.default_rng(5)
    keys = g.integers(-3, 3, size=5000).astype(np.int32)
    vals = np.arange(5000, dtype=np.int64) * 7 + 1
    k2, v2 = oracle.sort_pairs(keys, vals)
    assert np.array_equal(k2, np.sort(keys, kind="stable"))
    assert np.array_equal(v2, vals[np.argsort(keys, kind="stable")])
    assert np.array_equal(oracle.argsort(keys, np.int32), np.argsort(keys, kind="stable").astype(np.int32))


# --------------------------------------------------------------------------
# Radix steps
# --------------------------------------------------------------------------
def test_pass_counts_match_paper(golden):
    for dt, bits, passes in golden("radix_passes.txt"):
        assert oracle.pass_count(np.dtype(dt), int(bits)) == int(passes)


@pytest.mark.parametrize("bits", [4, 5, 8, 11, 12])
def test_histogram_uint32_equals_bincount(bits):
    x = workloads.uniform(np.uint32, 40_000, bits)
    h = oracle.digit_histogram(x, bits)
    for p in range(h.shape[0]):
        d = (x.astype(np.uint64) >> np.uint64(p * bits)) & np.uint64((1 << bits) - 1)
        assert np.array_equal(h[p], np.bincount(d.astype(np.int64), minlength=1 << bits).astype(np.uint64))


def test_histogram_int32_equals_xor_masked_uint32():
    """The paper's XOR-0x80000000 form (Sec. 4, Algorithm 4) against the oracle's own offset form."""
    x = workloads.uniform(np.int32, 40_000, 3)
    flipped = x.view(np.uint32) ^ np.uint32(0x80000000)
    assert np.array_equal(oracle.digit_histogram(x, 8), oracle.digit_histogram(flipped, 8))
    x64 = workloads.uniform(np.int64, 40_000, 3)
    flipped64 = x64.view(np.uint64) ^ np.uint64(0x8000000000000000)
    h = oracle.digit_histogram(x64, 8)
    for p in range(8):
        d = (flipped64 >> np.uint64(8 * p)) & np.uint64(255)
        assert np.array_equal(h[p], np.bincount(d.astype(np.int64), minlength=256).astype(np.uint64))


def test_digit_bases_exclusive():
    h = np.array([[3, 0, 2, 5], [1, 1, 1, 7]], dtype=np.uint64)
    assert np.array_equal(oracle.digit_bases(h), np.array([[0, 3, 3, 5], [0, 1, 2, 3]], dtype=np.uint64))


@pytest.mark.parametrize("bits,shift", [(8, 0), (8, 8), (8, 24), (4, 28), (11, 22), (6, 30)])
def test_counting_pass_is_stable_sort_by_digit(bits, shift):
    x = workloads.uniform(np.uint32, 3000, shift + bits)
    digit = [(int(v) >> shift) & ((1 << bits) - 1) for v in x]
    expect = sorted(range(len(x)), key=lambda i: digit[i])  # Python's sort is stable
    assert oracle.counting_pass(x, shift, bits).tolist() == expect


@pytest.mark.parametrize("dt", ALL_DTYPES)
@pytest.mark.parametrize("bits", [4, 7, 8, 11, 12])
def test_lsd_passes_compose_to_the_stable_sort(dt, bits):
    """LSD correctness: stable passes from the lowest digit up give the stable sort."""
    g = np.random.default_rng(bits)
    keys = workloads.uniform(dt, 5000, bits)
    keys[g.integers(0, 5000, 800)] = keys[g.integers(0, 5000, 800)]  # duplicates
    cur = np.arange(keys.size)
    for p in range(oracle.pass_count(dt, bits)):
        cur = cur[oracle.counting_pass(keys[cur], p * bits, bits)]
    assert np.array_equal(cur, oracle.stable_perm(keys))


# --------------------------------------------------------------------------
# Mergesort steps
# --------------------------------------------------------------------------
@pytest.mark.parametrize("chunk", [1, 2, 3, 17, 64, 195])
def test_insertion_chunks_sorts_each_chunk(chunk):
    g = np.random.default_rng(chunk)
    x = g.integers(-20, 20, size=1000).astype(np.int32)
    perm = oracle.insertion_chunks(x, chunk)
    for lo in range(0, len(x), chunk):
        seg = list(range(lo, min(lo + chunk, len(x))))
        assert perm[lo:lo + len(seg)].tolist() == sorted(seg, key=lambda i: int(x[i]))


@pytest.mark.parametrize("run", [1, 2, 5, 64, 333, 999, 1000, 1500])
def test_merge_round_merges_pairs(run):
    g = np.random.default_rng(run)
    n = 1000
    x = g.integers(-10, 10, size=n).astype(np.int64)
    # make every run sorted (stably) first, with the library sort
    for lo in range(0, n, run):
        seg = x[lo:lo + run]
        x[lo:lo + run] = seg[np.argsort(seg, kind="stable")]
    perm = oracle.merge_round(x, run)
    for lo in range(0, n, 2 * run):
        seg = list(range(lo, min(lo + 2 * run, n)))
        assert perm[lo:lo + len(seg)].tolist() == sorted(seg, key=lambda i: int(x[i]))


@pytest.mark.parametrize("dt", ALL_DTYPES)
@pytest.mark.parametrize("chunk", [2, 3, 17, 195, 629, 2048])
def test_bottom_up_schedule_reaches_the_stable_sort(dt, chunk):
    """Mergesort schedule of Sec. 4, Algorithm 3: insertion chunks, then runs doubling from the chunk size."""
    g = np.random.default_rng(chunk)
    n = 6007
    keys = workloads.uniform(dt, n, chunk)
    keys[g.integers(0, n, 1500)] = keys[g.integers(0, n, 1500)]
    cur = oracle.insertion_chunks(keys, chunk)
    run = chunk
    while run < n:
        cur = cur[oracle.merge_round(keys[cur], run)]
        run *= 2
    assert np.array_equal(cur, oracle.stable_perm(keys))


# --------------------------------------------------------------------------
# Sampled and property checks
# --------------------------------------------------------------------------
def test_rank_of_matches_inverse_permutation():
    g = np.random.default_rng(1)
    x = g.integers(-5, 5, size=3000).astype(np.int32)
    expect = sorted(range(len(x)), key=lambda i: (int(x[i]), i))
    pos = {i: j for j, i in enumerate(expect)}
    for i in g.integers(0, len(x), 50):
        assert oracle.rank_of(x, int(i)) == pos[int(i)]


def test_first_unsorted():
    x = np.arange(100, dtype=np.int32)
    assert oracle.first_unsorted(x) == -1
    x[40], x[41] = x[41], x[40]
    assert oracle.first_unsorted(x) == 40
    f = np.array([-0.0, 0.0, 0.0], dtype=np.float32)
    assert oracle.first_unsorted(f) == -1
    assert oracle.first_unsorted(f[::-1].copy()) == 1  # +0.0 then -0.0 is out of order


# --------------------------------------------------------------------------
# Dispatch (host logic)
# --------------------------------------------------------------------------
def test_aps_branches_match_paper_table(golden):
    for n, t_np, a_code, is_int, expect in golden("aps_dispatch.txt"):
        got = oracle.aps_path(int(n), bool(int(is_int)), int(a_code), int(t_np), small_capacity=10**18,
                              radix_for_floats=False)
        assert got == expect, (n, t_np, a_code, is_int)


def test_aps_gpu_readings(golden):
    """The dispatch rule with the GPU library's readings (one-workgroup capacity, A_code 0, float keys),
    against a table written by hand from those readings."""
    rows = golden("aps_dispatch_gpu.txt")
    assert len(rows) >= 20
    for n, t_np, a_code, is_int, cap, rff, expect in rows:
        got = oracle.aps_path(int(n), bool(int(is_int)), int(a_code), int(t_np), small_capacity=int(cap),
                              radix_for_floats=bool(int(rff)))
        assert got == expect, (n, t_np, a_code, is_int, cap, rff)


def test_struct_roundtrip_sanity():
    # the float golden file's hex patterns are the standard encodings
    assert struct.unpack("<f", struct.pack("<I", 0x3FC00000))[0] == 1.5
    assert struct.unpack("<d", struct.pack("<Q", 0x3FF8000000000000))[0] == 1.5


# --------------------------------------------------------------------------
# Batches of arrays (segmented sort)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("dt", INT_DTYPES)
def test_segmented_sort_equals_numpy_per_segment(dt):
    """Each segment equals numpy's stable sort of that segment; keys outside the segments are untouched."""
    sizes = workloads.segment_sizes(300, seed=3, median=40, sigma=1.5, lo=0, hi=3000)
    offs = workloads.segment_offsets(sizes) + 5  # a gap before the first segment
    n = int(offs[-1]) + 7                        # and one after the last
    keys = workloads.uniform(dt, n, 11) % 97     # many equal keys
    got = oracle.segmented_sort(keys, offs)
    assert np.array_equal(got[:5], keys[:5]) and np.array_equal(got[offs[-1]:], keys[offs[-1]:])
    for b, e in zip(offs[:-1], offs[1:]):
        assert np.array_equal(got[b:e], np.sort(keys[b:e], kind="stable"))


def test_segmented_pairs_follow_numpy_stable_argsort():
    sizes = np.array([0, 1, 2, 17, 0, 300, 5, 1000, 3], dtype=np.int64)
    offs = workloads.segment_offsets(sizes)
    keys = workloads.distinct16(np.int64, int(offs[-1]), 4)
    vals = np.arange(keys.size, dtype=np.uint32) * 3 + 1
    ko, vo = oracle.segmented_sort_pairs(keys, vals, offs)
    for b, e in zip(offs[:-1], offs[1:]):
        p = np.argsort(keys[b:e], kind="stable")
        assert np.array_equal(ko[b:e], keys[b:e][p]) and np.array_equal(vo[b:e], vals[b:e][p])


def test_segmented_degenerate_cases():
    keys = workloads.uniform(np.float32, 500, 9)
    # one segment over everything: the plain sort
    assert np.array_equal(oracle.segmented_sort(keys, [0, 500]).view(np.uint32), oracle.sort(keys).view(np.uint32))
    # segments of one key, or none: unchanged
    assert np.array_equal(oracle.segmented_sort(keys, np.arange(501)).view(np.uint32), keys.view(np.uint32))
    assert np.array_equal(oracle.segmented_sort(keys, [250]).view(np.uint32), keys.view(np.uint32))
    with pytest.raises(ValueError):
        oracle.segmented_sort(keys, [0, 300, 200])
    with pytest.raises(ValueError):
        oracle.segmented_sort(keys, [0, 501])


def test_segment_sizes_recipe():
    """Log-normal sizes: the median and the spread of log sizes follow the parameters; clipping holds."""
    s = workloads.segment_sizes(100_000, seed=42)
    assert s.min() >= 16 and s.max() <= 4_000_000
    assert abs(np.median(s) / 2048 - 1) < 0.05
    inner = s[(s > 16) & (s < 4_000_000)]
    assert abs(np.std(np.log(inner)) - 2.0) < 0.1  # clipping trims the tails a little
    assert np.array_equal(workloads.segment_offsets([3, 0, 2]), [0, 3, 3, 5])


# ---------------------------------------------------------------- descending --
def _selection_desc(u):
    """O(n^2) reference: repeatedly take the largest order key, the earliest index among equals."""
    left = list(range(len(u)))
    out = []
    while left:
        best = left[0]
        for i in left[1:]:
            if u[i] > u[best]:
                best = i
        out.append(best)
        left.remove(best)
    return np.array(out, dtype=np.int64)


@pytest.mark.parametrize("dt", [np.int32, np.int64, np.uint32, np.float32, np.float64])
def test_descending_brute_force_small(dt):
    """Every sequence of length <= 5 over a 3-value alphabet (with ties): descending stable order."""
    import itertools

    if np.dtype(dt).kind == "f":
        alphabet = np.array([-0.0, 0.0, 1.5], dtype=dt)
    else:
        alphabet = np.array([0, 7, np.iinfo(dt).max], dtype=dt)
    for n in range(0, 6):
        for combo in itertools.product(range(3), repeat=n):
            keys = alphabet[list(combo)] if n else np.zeros(0, dtype=dt)
            u = oracle.order_keys(keys)
            assert np.array_equal(oracle.stable_perm(keys, descending=True), _selection_desc(list(u))), keys


def test_descending_matches_numpy_lexsort_for_ints():
    x = workloads.uniform(np.int32, 20_000, 5) % 301 - 150  # many ties, both signs
    idx = np.arange(x.size)
    want = np.lexsort((idx, -x.astype(np.int64)))  # primary: value descending; ties: index ascending
    assert np.array_equal(oracle.stable_perm(x, descending=True), want)
    y = workloads.uniform(np.int64, 20_000, 6)
    y[::3] = y[1]
    want = np.lexsort((np.arange(y.size), -(y.astype(np.float64))))  # distinct magnitudes apart from the ties
    got = oracle.stable_perm(y, descending=True)
    assert np.array_equal(y[got], y[want])
    ties = np.flatnonzero(y[got] == y[1])
    assert np.all(np.diff(got[ties]) > 0)  # equal keys in input order


def test_descending_is_reversed_ascending_for_distinct_keys():
    x = np.unique(workloads.uniform(np.float64, 5000, 7))
    x = x[workloads.rng(8).permutation(x.size)]
    assert np.array_equal(oracle.stable_perm(x, descending=True), oracle.stable_perm(x)[::-1])
    pairs_k, pairs_v = oracle.sort_pairs(x, np.arange(x.size), descending=True)
    assert np.array_equal(pairs_k.view(np.uint64), oracle.sort(x)[::-1].view(np.uint64))


def test_descending_segments():
    sizes = np.array([0, 1, 5, 300, 2], dtype=np.int64)
    offs = workloads.segment_offsets(sizes)
    keys = workloads.distinct16(np.int32, int(offs[-1]), 9)
    got = oracle.segmented_sort(keys, offs, descending=True)
    for b, e in zip(offs[:-1], offs[1:]):
        assert np.array_equal(got[b:e], np.sort(keys[b:e])[::-1])
