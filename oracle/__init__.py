"""Reference oracle for the EvoSort sort path -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The GPU library and its Python binding never do.

The heavy lifting is plain C in ``evosort_oracle.c`` (loaded through ctypes);
this module marshals numpy arrays and adds the host-side dispatch rule.

Every function returns results computed on the CPU from the definition of a
stable sort (see the C file's header):

* :func:`stable_perm`   -- the unique stable sorting permutation;
* :func:`sort`, :func:`sort_pairs`, :func:`argsort` -- results of the three
  library calls, obtained by gathering through that permutation;
* :func:`digit_histogram`, :func:`digit_bases`, :func:`counting_pass` -- the
  steps of one LSD radix pass (Sec. 4, Algorithms 4 and 5, the block-based LSD radix sort);
* :func:`insertion_chunks`, :func:`merge_round` -- the steps of the bottom-up
  mergesort (Sec. 4, Algorithm 3, the refined parallel mergesort);
* :func:`segmented_sort`, :func:`segmented_sort_pairs` -- a batch of arrays
  (segments of one buffer), each sorted on its own;
* :func:`rank_of`, :func:`first_unsorted` -- sampled and property checks for
  sizes the full host sort is too slow for;
* :func:`aps_path` -- which routine the adaptive partition sort picks
  (Sec. 4.3, Algorithm 6, AdaptivePartitionSort).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

# The oracle's own kind codes (see evosort_oracle.c).
_KINDS = {
    np.dtype(np.int32): 1,
    np.dtype(np.int64): 2,
    np.dtype(np.uint32): 3,
    np.dtype(np.float32): 4,
    np.dtype(np.float64): 5,
}

_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _build

        _build.build()
    lib = ctypes.CDLL(_LIB_PATH)
    i64 = ctypes.c_int64
    vp = ctypes.c_void_p
    ci = ctypes.c_int
    lib.oracle_order_keys.argtypes = [ci, vp, i64, vp]
    lib.oracle_stable_perm.argtypes = [ci, vp, i64, vp]
    lib.oracle_stable_perm_dir.argtypes = [ci, vp, i64, ci, vp]
    lib.oracle_digit_histogram.argtypes = [ci, vp, i64, ci, vp]
    lib.oracle_counting_pass.argtypes = [ci, vp, i64, ci, ci, vp]
    lib.oracle_insertion_chunks.argtypes = [ci, vp, i64, i64, vp]
    lib.oracle_merge_round.argtypes = [ci, vp, i64, i64, vp]
    lib.oracle_rank_of.argtypes = [ci, vp, i64, i64, vp]
    lib.oracle_first_unsorted.argtypes = [ci, vp, i64]
    lib.oracle_first_unsorted.restype = i64
    for f in (lib.oracle_order_keys, lib.oracle_stable_perm, lib.oracle_digit_histogram,
              lib.oracle_counting_pass, lib.oracle_insertion_chunks, lib.oracle_merge_round,
              lib.oracle_rank_of):
        f.restype = ci
    _lib = lib
    return lib


def _kind(a: np.ndarray) -> int:
    try:
        return _KINDS[a.dtype]
    except KeyError:
        raise TypeError(f"oracle: unsupported key dtype {a.dtype}") from None


def _contig(a: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(a)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p) if a.size else None


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def key_bytes(dtype) -> int:
    return np.dtype(dtype).itemsize


def order_keys(keys: np.ndarray) -> np.ndarray:
    """Order keys as uint64: a < b in the key order iff order_keys(a) < order_keys(b)."""
    keys = _contig(keys)
    out = np.empty(keys.size, dtype=np.uint64)
    _check(_load().oracle_order_keys(_kind(keys), _ptr(keys), keys.size, _ptr(out)), "order_keys")
    return out


def stable_perm(keys: np.ndarray, descending: bool = False) -> np.ndarray:
    """The unique stable sorting permutation (int64) of ``keys``: ascending, or descending with equal keys
    still in input order."""
    keys = _contig(keys)
    perm = np.empty(keys.size, dtype=np.int64)
    _check(_load().oracle_stable_perm_dir(_kind(keys), _ptr(keys), keys.size, 1 if descending else 0, _ptr(perm)),
           "stable_perm")
    return perm


def sort(keys: np.ndarray, descending: bool = False) -> np.ndarray:
    """Result of a keys-only sort: keys gathered through the stable permutation."""
    keys = _contig(keys)
    return keys[stable_perm(keys, descending)]


def sort_pairs(keys: np.ndarray, vals: np.ndarray, descending: bool = False):
    """Result of a key-value sort: (keys, values) gathered through the stable permutation."""
    keys = _contig(keys)
    vals = _contig(vals)
    if vals.shape[0] != keys.shape[0]:
        raise ValueError("keys and values differ in length")
    perm = stable_perm(keys, descending)
    return keys[perm], vals[perm]


def argsort(keys: np.ndarray, index_dtype=np.int64, descending: bool = False) -> np.ndarray:
    """Result of an argsort: the stable permutation in the requested index type."""
    return stable_perm(keys, descending).astype(index_dtype)


def _segments(offsets, n: int):
    offsets = np.asarray(offsets, dtype=np.int64)
    if offsets.ndim != 1 or offsets.size < 1:
        raise ValueError("offsets needs nseg + 1 entries")
    if np.any(np.diff(offsets) < 0) or offsets[0] < 0 or offsets[-1] > n:
        raise ValueError("offsets must be non-decreasing within [0, n]")
    return zip(offsets[:-1].tolist(), offsets[1:].tolist())


def segmented_sort(keys: np.ndarray, offsets, descending: bool = False) -> np.ndarray:
    """Result of a batched segmented sort: every segment keys[offsets[i]:offsets[i+1]]
    replaced by its own stable sort; keys outside the segments are unchanged."""
    keys = _contig(keys)
    out = keys.copy()
    for b, e in _segments(offsets, keys.size):
        if e - b > 1:
            out[b:e] = sort(keys[b:e], descending)
    return out


def segmented_sort_pairs(keys: np.ndarray, vals: np.ndarray, offsets, descending: bool = False):
    """Key-value version of :func:`segmented_sort` (values travel with their keys)."""
    keys = _contig(keys)
    vals = _contig(vals)
    if vals.shape[0] != keys.shape[0]:
        raise ValueError("keys and values differ in length")
    ko, vo = keys.copy(), vals.copy()
    for b, e in _segments(offsets, keys.size):
        if e - b > 1:
            perm = stable_perm(keys[b:e], descending)
            ko[b:e] = keys[b:e][perm]
            vo[b:e] = vals[b:e][perm]
    return ko, vo


def pass_count(dtype, digit_bits: int) -> int:
    """Number of digit positions covering a key of ``dtype`` at ``digit_bits`` bits each."""
    bits = 8 * key_bytes(dtype)
    return (bits + digit_bits - 1) // digit_bits


def digit_histogram(keys: np.ndarray, digit_bits: int) -> np.ndarray:
    """(passes, 2**digit_bits) uint64 counts of every digit of every pass."""
    keys = _contig(keys)
    passes = pass_count(keys.dtype, digit_bits)
    hist = np.zeros((passes, 1 << digit_bits), dtype=np.uint64)
    _check(_load().oracle_digit_histogram(_kind(keys), _ptr(keys), keys.size, digit_bits, _ptr(hist)),
           "digit_histogram")
    return hist


def digit_bases(hist: np.ndarray) -> np.ndarray:
    """Exclusive prefix sums of each pass's histogram: the first output slot of each digit."""
    hist = np.asarray(hist, dtype=np.uint64)
    inclusive = np.cumsum(hist, axis=1, dtype=np.uint64)
    return inclusive - hist


def counting_pass(keys: np.ndarray, shift: int, digit_bits: int) -> np.ndarray:
    """Permutation of one stable counting pass on the digit at bit offset ``shift``."""
    keys = _contig(keys)
    perm = np.empty(keys.size, dtype=np.int64)
    _check(_load().oracle_counting_pass(_kind(keys), _ptr(keys), keys.size, shift, digit_bits, _ptr(perm)),
           "counting_pass")
    return perm


def insertion_chunks(keys: np.ndarray, chunk: int) -> np.ndarray:
    """Permutation that insertion-sorts every chunk of ``chunk`` keys on its own."""
    keys = _contig(keys)
    perm = np.empty(keys.size, dtype=np.int64)
    _check(_load().oracle_insertion_chunks(_kind(keys), _ptr(keys), keys.size, chunk, _ptr(perm)),
           "insertion_chunks")
    return perm


def merge_round(keys: np.ndarray, run: int) -> np.ndarray:
    """Permutation of one merge round over pairs of adjacent sorted runs of length ``run``."""
    keys = _contig(keys)
    perm = np.empty(keys.size, dtype=np.int64)
    _check(_load().oracle_merge_round(_kind(keys), _ptr(keys), keys.size, run, _ptr(perm)), "merge_round")
    return perm


def rank_of(keys: np.ndarray, i: int) -> int:
    """Output position of input element ``i`` under the stable sort (one O(n) pass)."""
    keys = _contig(keys)
    r = ctypes.c_int64(-1)
    _check(_load().oracle_rank_of(_kind(keys), _ptr(keys), keys.size, int(i), ctypes.byref(r)), "rank_of")
    return int(r.value)


def first_unsorted(keys: np.ndarray) -> int:
    """First j with keys[j] > keys[j+1] in the key order, or -1."""
    keys = _contig(keys)
    return int(_load().oracle_first_unsorted(_kind(keys), _ptr(keys), keys.size))


# Routine codes of the adaptive partition sort (Sec. 4.2: A_code 3 is the
# mergesort, A_code 4 the LSD radix sort).
A_MERGE = 3
A_RADIX = 4


def aps_path(n: int, integer_keys: bool, a_code: int, t_fallback: int, small_capacity: int,
             radix_for_floats: bool = True) -> str:
    """Routine chosen by the adaptive partition sort (Sec. 4.3, Algorithm 6, AdaptivePartitionSort).

    The paper's rule: below the library-sort threshold use the small-array
    sort; else the LSD radix sort when A_code is 4 and the keys are integers;
    else the refined mergesort (A_code 3, and every other code, in the paper).

    Readings for the GPU library: the small-array sort is one workgroup, so the
    branch also needs n to fit in one workgroup (``small_capacity`` is the
    largest n it takes); float
    keys take the radix branch too when ``radix_for_floats`` (their keys are
    mapped to unsigned integers); A_code 0 means "automatic" and picks the radix
    sort, which the paper's tuner chose at every size.
    """
    if n < t_fallback and n <= small_capacity:
        return "small"
    if a_code in (0, A_RADIX) and (integer_keys or radix_for_floats):
        return "radix"
    return "merge"
