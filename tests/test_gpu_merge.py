"""GPU parity of the mergesort steps against the oracle's steps.

Rows: the block sort (Sec. 4, Algorithm 3: chunks of T_ins insertion-sorted,
then merged pairwise up to the block size) and one merge round (the same
algorithm's loop body, with ties to the left run and a trailing run copied).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


def _oracle_block_sort(keys, t_ins, block):
    """Alg. 3 schedule restricted to blocks: insertion chunks, then merges with run < block."""
    cur = oracle.insertion_chunks(keys, t_ins)
    run = t_ins
    while run < block:
        # merges never cross a block boundary because block is t_ins * 2^m
        cur = cur[oracle.merge_round(keys[cur], run)]
        run *= 2
    return cur


# T_ins 1, 2, 4 and 8 on full blocks is the register path: each thread's 8
# records sorted and merged up to one wave's 512 in registers, the rest of
# the levels in LDS; the other values rank chunks and merge in LDS only.
@pytest.mark.parametrize("dt", [np.uint32, np.int32, np.float32, np.int64, np.float64])
@pytest.mark.parametrize("t_ins", [1, 2, 3, 4, 8, 195, 2048])
@pytest.mark.parametrize("n", [1, 5, 4096, 10_000])
@pytest.mark.parametrize("vals_dtype", [None, np.int32, np.int64])
def test_block_sort(dt, t_ins, n, vals_dtype):
    es = require_gpu()
    keys = workloads.uniform(dt, n, t_ins + n)
    keys[::3] = keys[0]
    vals = None if vals_dtype is None else (np.arange(n) + 100).astype(vals_dtype)
    p = es.default_params(algo=es.ALGO_MERGE, insertion_threshold=t_ins)
    k, v, run = es.merge_block_sort(to_dev(keys), None if vals is None else to_dev(vals), params=p)
    assert run % t_ins == 0 and (run // t_ins) & (run // t_ins - 1) == 0  # t_ins * 2^m
    perm = _oracle_block_sort(keys, t_ins, run)
    assert_bits_equal(to_np(k), keys[perm], "block sort keys")
    if vals is not None:
        assert_bits_equal(to_np(v), vals[perm], "block sort values")


@pytest.mark.parametrize("dt", [np.uint32, np.int32, np.float32, np.int64, np.float64])
@pytest.mark.parametrize("run", [1, 3, 100, 2048, 4096, 5000, 30_000])
def test_merge_round(dt, run):
    es = require_gpu()
    n = 70_001
    g = np.random.default_rng(run)
    keys = workloads.uniform(dt, n, run)
    keys[g.integers(0, n, n // 3)] = keys[g.integers(0, n, n // 3)]
    # sorted runs of length `run` (made with the oracle)
    perm0 = np.concatenate([lo + oracle.stable_perm(keys[lo:lo + run]) for lo in range(0, n, run)])
    keys = keys[perm0]
    vals = np.arange(n, dtype=np.int32) * 5
    k, v = es.merge_round(to_dev(keys), to_dev(vals), run=run)
    perm = oracle.merge_round(keys, run)
    assert_bits_equal(to_np(k), keys[perm], f"merge round run={run}")
    assert_bits_equal(to_np(v), vals[perm], f"merge round values run={run}")
