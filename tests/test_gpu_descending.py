"""Descending order on the GPU against the oracle's descending stable sort, element by element:
every key type, every routine (radix, mergesort, one-workgroup), keys / pairs / argsort, the step
entry points' invariance and the batched sort."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

DTYPES = [np.int32, np.int64, np.uint32, np.float32, np.float64]
ROUTINES = {"radix": dict(algo=4, fallback_threshold=0), "merge": dict(algo=3, fallback_threshold=0),
            "small": dict()}


def _keys(dt, n, seed):
    if np.dtype(dt).kind == "f":
        k = workloads.float_mix(dt, n, seed)
        k[: min(n, 16)] = np.resize(workloads.float_edges(dt), min(n, 16))
        return k
    k = workloads.uniform(dt, n, seed)
    k[::5] = k[1]  # ties: input order must survive
    return k


@pytest.mark.parametrize("routine", list(ROUTINES))
@pytest.mark.parametrize("dt", DTYPES)
def test_descending_sort_pairs_argsort(dt, routine):
    es = require_gpu()
    import torch

    n = 3000 if routine == "small" else 150_001
    keys = _keys(dt, n, 21)
    p = es.default_params(descending=1, **ROUTINES[routine])
    assert es.plan(es.OP_SORT, es.dtype_code(to_dev(keys[:1]).dtype), n, 0, p)["path_name"] == routine
    perm = oracle.stable_perm(keys, descending=True)
    k = to_dev(keys)
    assert_bits_equal(to_np(es.sort(k, params=p)), keys[perm], f"descending sort {routine}")
    vals = np.arange(n, dtype=np.int64) * 3 + 1
    ko, vo = es.sort_pairs(k, to_dev(vals), params=p)
    assert_bits_equal(to_np(ko), keys[perm], "descending pairs keys")
    assert np.array_equal(to_np(vo), vals[perm]), "descending pairs values"
    idx = to_np(es.argsort(k, index_dtype=torch.int32, params=p))
    assert np.array_equal(idx, perm.astype(np.int32)), "descending argsort"


@pytest.mark.parametrize("bits", [4, 8, 11])
def test_descending_invariant_over_digit_width(bits):
    es = require_gpu()
    keys = workloads.distinct16(np.int64, 70_000, 3)
    p = es.default_params(descending=1, algo=4, fallback_threshold=0, digit_bits=bits)
    got = to_np(es.sort(to_dev(keys), params=p))
    assert_bits_equal(got, oracle.sort(keys, descending=True), f"descending d={bits}")


def test_descending_in_place_and_ascending_unchanged():
    es = require_gpu()
    keys = workloads.uniform(np.float32, 99_999, 4)
    k = to_dev(keys)
    es.sort(k, params=es.default_params(descending=1), out=k)
    assert_bits_equal(to_np(k), oracle.sort(keys, descending=True), "descending in place")
    assert_bits_equal(to_np(es.sort(to_dev(keys))), oracle.sort(keys), "ascending default")


@pytest.mark.parametrize("dt", [np.uint32, np.float64])
def test_descending_segmented(dt):
    es = require_gpu()
    sizes = workloads.segment_sizes(2000, 8, median=400.0, sigma=2.0, lo=0, hi=120_000)
    offs = workloads.segment_offsets(sizes)
    keys = _keys(dt, int(offs[-1]), 9)
    p = es.default_params(descending=1)
    got = to_np(es.segmented_sort(to_dev(keys), to_dev(offs), params=p))
    assert_bits_equal(got, oracle.segmented_sort(keys, offs, descending=True), "descending segmented")


def test_descending_server():
    es = require_gpu()
    reqs = [_keys(np.int32, int(n), 30 + i) for i, n in enumerate([10, 5000, 70_000, 300_000])]
    with es.Server(hbm_budget_bytes=256 << 20, params=es.default_params(descending=1)) as srv:
        ids = [srv.submit(to_dev(k)) for k in reqs]
        for rid, k in zip(ids, reqs):
            assert_bits_equal(to_np(srv.result(rid)), oracle.sort(k, descending=True), "descending served")
            srv.release(rid)


def test_descending_rejects_bad_flag():
    es = require_gpu()
    p = es.default_params()
    p.descending = 2
    with pytest.raises(es.EvosortError):
        es.sort(to_dev(np.arange(10, dtype=np.int32)), params=p)
