"""Every default tile shape of the radix passes for large arrays, element by element against the oracle.

Above 2^21 keys the library takes its large-array tile per (key bytes, value
bytes): 768 x 24 for 4-byte keys alone or with 4-byte values, 512 x 24 for
4-byte keys with 8-byte values and for 8-byte keys with 4-byte values,
768 x 12 for 8-byte keys alone (the kernel of the 1e9 int64 benchmark sort),
512 x 16 for 8-byte keys with 8-byte values (Sec. 4, Algorithms 4 and 5: one
stable pass per digit).  Each shape runs with 32-bit look-back words (every
n < 2^30) and with 64-bit ones (every n >= 2^30, reached here at a small size
through EVOSORT_DEBUG_WIDE_STATUS), for keys only, key-value pairs with 4- and
8-byte values and argsort with int32 and int64 indices, at a size that spans
hundreds of tiles and ends in a ragged tile.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

N = (1 << 22) + 12345
# the default at N keys (pairs with an 8-byte word take their mid-size tiles below 2^26 keys), and the
# large-array tiles those pairs take above 2^26 keys, checked here at N by asking for them
EXPECTED_TILE = {(4, 0): (768, 24), (4, 4): (768, 24), (4, 8): (768, 16),
                 (8, 0): (768, 12), (8, 4): (768, 16), (8, 8): (768, 12)}
LARGE_TILE = {(4, 0): (768, 24), (4, 4): (768, 24), (4, 8): (512, 24),
              (8, 0): (768, 12), (8, 4): (512, 24), (8, 8): (512, 16)}
_CACHE = {}


def _case(dt):
    """Keys with ties (every 5th key repeats one value, a run of equal keys) and, for floats, the edge mix;
    the oracle's stable permutation of them."""
    if dt not in _CACHE:
        if np.dtype(dt).kind == "f":
            keys = workloads.float_mix(dt, N, 31)
        else:
            keys = workloads.uniform(dt, N, 31)
        keys[::5] = keys[7]
        keys[1000:5000] = keys[3]
        _CACHE.clear()
        _CACHE[dt] = (keys, oracle.stable_perm(keys))
    return _CACHE[dt]


@pytest.mark.parametrize("tiles", ["default", "large"])
@pytest.mark.parametrize("wide", [False, True], ids=["status32", "status64"])
@pytest.mark.parametrize("dt", [np.int32, np.float32, np.uint32, np.int64, np.float64])
def test_default_large_array_tiles(dt, wide, tiles):
    """Keys only, pairs with 4- and 8-byte values and argsort with 32- and 64-bit indices on the default tiles
    at N keys, and on the large-array tiles where those differ, element by element against the oracle."""
    import torch

    es = require_gpu()
    keys, perm = _case(dt)
    kb = np.dtype(dt).itemsize
    code = es.dtype_code(torch.from_numpy(keys[:1]).dtype)
    flags = es.DEBUG_WIDE_STATUS if wide else 0
    table = EXPECTED_TILE if tiles == "default" else LARGE_TILE

    # A_code 4: the hand-coded tiles (the automatic choice may take the tuner's routine at some sizes; those
    # sorts are checked with the tuner's tests)
    def params(vb):
        if tiles == "default":
            return es.default_params(algo=es.ALGO_RADIX, debug_flags=flags)
        t, i = LARGE_TILE[(kb, vb)]
        return es.default_params(algo=es.ALGO_RADIX, debug_flags=flags, block_threads=t, items_per_thread=i)

    def runs(vb):  # the large-array pass checks only the tiles the default does not already take
        return tiles == "default" or LARGE_TILE[(kb, vb)] != EXPECTED_TILE[(kb, vb)]

    for op, vb in ((es.OP_SORT, 0), (es.OP_SORT_PAIRS, 4), (es.OP_SORT_PAIRS, 8), (es.OP_ARGSORT, 4),
                   (es.OP_ARGSORT, 8)):
        info = es.plan(op, code, N, vb, params(vb))
        assert info["path_name"] == "radix"
        assert (info["block_threads"], info["items_per_thread"]) == table[(kb, vb)], (op, vb, info)
        assert info["status_bytes"] == (8 if wide else 4)
        assert info["tiles"] > 200
    if not any(runs(vb) for vb in (0, 4, 8)):
        return
    want = keys[perm]
    k = to_dev(keys)
    if runs(0):
        assert_bits_equal(to_np(es.sort(k, params=params(0), check=True)), want, "keys")
    if runs(4):
        v4 = (np.arange(N, dtype=np.int64) * 7 + 3).astype(np.int32)
        k4, o4 = es.sort_pairs(k, to_dev(v4), params=params(4), check=True)
        assert_bits_equal(to_np(k4), want, "pairs(4) keys")
        assert_bits_equal(to_np(o4), v4[perm], "pairs(4) values")
        assert np.array_equal(to_np(es.argsort(k, index_dtype=torch.int32, params=params(4), check=True)),
                              perm.astype(np.int32)), "argsort int32"
    if runs(8):
        v8 = (np.arange(N, dtype=np.int64) * 2654435761) % (2 ** 61)
        k8, o8 = es.sort_pairs(k, to_dev(v8), params=params(8), check=True)
        assert_bits_equal(to_np(k8), want, "pairs(8) keys")
        assert_bits_equal(to_np(o8), v8[perm], "pairs(8) values")
        assert np.array_equal(to_np(es.argsort(k, index_dtype=torch.int64, params=params(8), check=True)),
                              perm), "argsort int64"


@pytest.mark.parametrize("wide", [False, True], ids=["status32", "status64"])
def test_default_tiles_descending_and_in_place(wide):
    """The 8-byte default tile with descending order, sorted in place (odd pass counts need no copy here:
    8 passes)."""
    es = require_gpu()
    keys, _ = _case(np.int64)
    p = es.default_params(descending=1, debug_flags=es.DEBUG_WIDE_STATUS if wide else 0)
    k = to_dev(keys)
    es.sort(k, params=p, out=k, check=True)
    assert_bits_equal(to_np(k), oracle.sort(keys, descending=True), "descending in place")


@pytest.mark.parametrize("dt, n", [(np.int32, 2_462_681), (np.int32, 3_427_305), (np.uint32, 4_043_198),
                                   (np.float32, 4_769_769), (np.int32, 10_000_007)])
def test_cu_rounded_tiles_match_oracle(dt, n):
    """The tiles the CU-rounding rule picks between 2^21 and 2^26 keys (768 x 16, 768 x 20, 1024 x 16,
    1024 x 20): keys only, pairs with 4-byte values and argsort with 32-bit indices, element by element
    against the oracle, ties included."""
    import torch

    es = require_gpu()
    keys = workloads.float_mix(dt, n, 17) if np.dtype(dt).kind == "f" else workloads.uniform(dt, n, 17)
    keys[::7] = keys[3]
    perm = oracle.stable_perm(keys)
    k = to_dev(keys)
    p = es.default_params(algo=es.ALGO_RADIX)
    code = es.dtype_code(k.dtype)
    shapes = {(es.plan(op, code, n, vb, p)["block_threads"], es.plan(op, code, n, vb, p)["items_per_thread"])
              for op, vb in ((es.OP_SORT, 0), (es.OP_SORT_PAIRS, 4))}
    assert shapes & {(768, 16), (768, 20), (1024, 16), (1024, 20)}, shapes
    assert_bits_equal(to_np(es.sort(k, params=p, check=True)), keys[perm], "keys")
    v = (np.arange(n, dtype=np.int64) * 5 + 1).astype(np.int32)
    ko, vo = es.sort_pairs(k, to_dev(v), params=p, check=True)
    assert_bits_equal(to_np(ko), keys[perm], "pairs keys")
    assert_bits_equal(to_np(vo), v[perm], "pairs values")
    assert np.array_equal(to_np(es.argsort(k, index_dtype=torch.int32, params=p, check=True)), perm), "argsort"


@pytest.mark.parametrize("dt, n", [(np.int64, 524_289), (np.float64, 1_000_003), (np.int64, 2_097_152)])
def test_mid_size_keys_take_768x12(dt, n):
    """Keys above 2^19 keys sort on the 768 x 12 tile up to 2^21 keys (and 8-byte keys without values above),
    element by element like the oracle; pairs with 8-byte values take it too."""
    es = require_gpu()
    keys = workloads.float_mix(dt, n, 23) if np.dtype(dt).kind == "f" else workloads.uniform(dt, n, 23)
    keys[::9] = keys[2]
    k = to_dev(keys)
    p = es.default_params(algo=es.ALGO_RADIX)
    code = es.dtype_code(k.dtype)
    info = es.plan(es.OP_SORT, code, n, 0, p)
    assert (info["block_threads"], info["items_per_thread"]) == (768, 12)
    pairs = es.plan(es.OP_SORT_PAIRS, code, n, 8, p)
    assert (pairs["block_threads"], pairs["items_per_thread"]) == (768, 12)
    assert_bits_equal(to_np(es.sort(k, params=p, check=True)), oracle.sort(keys), "keys")
    v = np.arange(n, dtype=np.int64) * 11 - 3
    ko, vo = es.sort_pairs(k, to_dev(v), params=p, check=True)
    perm = oracle.stable_perm(keys)
    assert_bits_equal(to_np(ko), keys[perm], "pairs keys")
    assert_bits_equal(to_np(vo), v[perm], "pairs values")


@pytest.mark.parametrize("kdt, vb, shape", [(np.int32, 8, (768, 16)), (np.float64, 4, (768, 16)),
                                            (np.int64, 8, (768, 12))])
def test_mid_size_pairs_with_an_8_byte_word(kdt, vb, shape):
    """Pairs with an 8-byte key or value between 2^21 and 2^26 keys sort on their mid-size tile (768 x 16 with
    one 8-byte word, 768 x 12 with two), and argsort with 64-bit indices likewise, element by element against
    the oracle."""
    import torch

    es = require_gpu()
    n = 3_000_017
    keys = workloads.float_mix(kdt, n, 29) if np.dtype(kdt).kind == "f" else workloads.uniform(kdt, n, 29)
    keys[::6] = keys[1]
    perm = oracle.stable_perm(keys)
    k = to_dev(keys)
    p = es.default_params(algo=es.ALGO_RADIX)
    code = es.dtype_code(k.dtype)
    info = es.plan(es.OP_SORT_PAIRS, code, n, vb, p)
    assert (info["block_threads"], info["items_per_thread"]) == shape
    v = (np.arange(n, dtype=np.int64) * 3 + 7)
    v = v.astype(np.int32) if vb == 4 else v
    ko, vo = es.sort_pairs(k, to_dev(v), params=p, check=True)
    assert_bits_equal(to_np(ko), keys[perm], "pairs keys")
    assert_bits_equal(to_np(vo), v[perm], "pairs values")
    assert np.array_equal(to_np(es.argsort(k, index_dtype=torch.int64, params=p, check=True)), perm), "argsort"
