"""GPU parity of the radix steps, each against the oracle's step of the same name.

Rows: the all-pass digit histogram and its digit bases (Sec. 4, Algorithm 4,
histogram and prefix-sum steps), and one stable LSD pass (the same algorithm's
offset and placement steps), for every key type, several digit widths, sizes
spanning several tiles with a ragged last tile, and skewed inputs.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

DTYPES = [np.uint32, np.int32, np.float32, np.int64, np.float64]
SIZES = [1, 2, 4095, 4096, 4097, 3 * 4096 + 17, 100_003]


def _keys(dt, n, seed, dist="uniform"):
    if dist == "uniform":
        return workloads.uniform(dt, n, seed)
    if dist == "few":
        g = np.random.default_rng(seed)
        pool = workloads.uniform(dt, 3, seed + 1)
        return pool[g.integers(0, 3, size=n)]
    if dist == "equal":
        return np.full(n, workloads.uniform(dt, 1, seed)[0], dtype=dt)
    raise ValueError(dist)


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("bits", [4, 8, 11, 12])
@pytest.mark.parametrize("n", [0, 1, 4097, 100_003])
def test_histogram_and_bases(dt, bits, n):
    es = require_gpu()
    keys = _keys(dt, n, bits * 7 + n)
    hist, bases = es.radix_histogram(to_dev(keys), bits)
    want = oracle.digit_histogram(keys, bits)
    assert np.array_equal(to_np(hist).view(np.uint64), want)
    assert np.array_equal(to_np(bases).view(np.uint64), oracle.digit_bases(want))


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", SIZES)
@pytest.mark.parametrize("dist", ["uniform", "few", "equal"])
def test_one_pass_equals_counting_pass(dt, n, dist):
    es = require_gpu()
    keys = _keys(dt, n, n + 3, dist)
    vals = np.arange(n, dtype=np.int64) * 3 + 1
    passes = oracle.pass_count(dt, 8)
    for p in sorted({0, 1, passes - 1}):
        perm = oracle.counting_pass(keys, 8 * p, 8)
        k, v = es.radix_pass(to_dev(keys), to_dev(vals), pass_index=p)
        assert_bits_equal(to_np(k), keys[perm], f"pass {p} keys")
        assert_bits_equal(to_np(v), vals[perm], f"pass {p} values")
        k0, _ = es.radix_pass(to_dev(keys), None, pass_index=p)
        assert_bits_equal(to_np(k0), keys[perm], f"pass {p} keys-only")


@pytest.mark.parametrize("bits", [4, 5, 6, 7, 9, 10, 11, 12])
def test_one_pass_other_digit_widths(bits):
    es = require_gpu()
    n = 3 * 4096 + 1234
    for dt in (np.uint32, np.int64):
        keys = _keys(dt, n, bits)
        p = oracle.pass_count(dt, bits) - 1  # the (possibly narrower) top digit
        for pi in (0, p):
            perm = oracle.counting_pass(keys, bits * pi, bits)
            params = es.default_params(digit_bits=bits)
            k, _ = es.radix_pass(to_dev(keys), None, pass_index=pi, params=params)
            assert_bits_equal(to_np(k), keys[perm], f"bits {bits} pass {pi} {dt}")


@pytest.mark.parametrize("shape", [(256, 8), (256, 12), (256, 16), (256, 24), (256, 32), (512, 8), (512, 16)])
def test_one_pass_tile_shapes(shape):
    es = require_gpu()
    n = 5 * shape[0] * shape[1] + 77
    keys = _keys(np.uint32, n, shape[1])
    vals = np.arange(n, dtype=np.int32)
    params = es.default_params(block_threads=shape[0], items_per_thread=shape[1])
    perm = oracle.counting_pass(keys, 8, 8)
    k, v = es.radix_pass(to_dev(keys), to_dev(vals), pass_index=1, params=params)
    assert_bits_equal(to_np(k), keys[perm], f"shape {shape}")
    assert_bits_equal(to_np(v), vals[perm], f"shape {shape} values")
