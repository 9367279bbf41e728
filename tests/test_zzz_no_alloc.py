"""The allocation-free sort (evosort_sort_noalloc) against evosort_sort and the oracle.

Two calls in a row on the device's shared scratch array -- the second with a
smaller input, so it runs over what the first left there -- must each give
the bytes evosort_sort gives (the unique stable sort, element by element);
likewise on the small-array and mergesort routines, in place, and inside a
captured HIP graph replayed with new inputs.  A size whose scratch exceeds
the array is refused with EVOSORT_ERR_TEMP_TOO_SMALL and writes nothing.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


def _keys(dt, n, seed):
    keys = workloads.float_mix(dt, n, seed) if np.dtype(dt).kind == "f" else workloads.uniform(dt, n, seed)
    keys[::3] = keys[1]  # ties
    return keys


@pytest.mark.parametrize("dt", [np.int32, np.uint32, np.float32, np.int64, np.float64])
def test_two_calls_in_a_row_match_the_allocating_sort(dt):
    es = require_gpu()
    for n in (3_000_001, 200_003):  # the second call is smaller and reuses the array
        keys = _keys(dt, n, 20 + n % 7)
        code = es.dtype_code(to_dev(keys[:1]).dtype)
        assert es.plan(es.OP_SORT, code, n)["temp_bytes"] <= es.NOALLOC_SCRATCH_BYTES
        k = to_dev(keys)
        want = to_np(es.sort(k, check=True))
        got = to_np(es.sort_noalloc(k))
        assert_bits_equal(got, want, f"noalloc vs sort, n={n}")
        assert_bits_equal(got, oracle.sort(keys), f"noalloc vs oracle, n={n}")


def test_every_routine_and_in_place():
    es = require_gpu()
    keys = _keys(np.int32, 150_001, 3)
    k = to_dev(keys)
    want = oracle.sort(keys)
    for params in (es.default_params(), es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0),
                   es.default_params(digit_bits=11, fallback_threshold=0)):
        assert_bits_equal(to_np(es.sort_noalloc(k, params=params)), want, f"{params}")
    small = keys[:5000]
    assert_bits_equal(to_np(es.sort_noalloc(to_dev(small))), oracle.sort(small), "small-array routine")
    inplace = to_dev(keys)
    es.sort_noalloc(inplace, out=inplace, params=es.default_params(digit_bits=11, fallback_threshold=0))
    assert_bits_equal(to_np(inplace), want, "in place, odd pass count")


def test_oversized_input_is_refused():
    import torch

    es = require_gpu()
    n = 20_000_000  # int32 keys: about 80 MB of scratch
    assert es.plan(es.OP_SORT, es.INT32, n)["temp_bytes"] > es.NOALLOC_SCRATCH_BYTES
    k = torch.zeros(n, dtype=torch.int32, device="cuda")
    out = torch.full_like(k, 7)
    with pytest.raises(es.EvosortError) as e:
        es.sort_noalloc(k, out=out)
    assert e.value.status == es.ERR_TEMP_TOO_SMALL
    torch.cuda.synchronize()
    assert bool((out == 7).all().item()), "a refused call wrote nothing"


def test_graph_capture_replays():
    """The call captured in a HIP graph (nothing to allocate, no memset) and replayed with new inputs."""
    import torch

    es = require_gpu()
    n = 400_001
    keys_dev = torch.empty(n, dtype=torch.int64, device="cuda")
    out = torch.empty_like(keys_dev)
    first = _keys(np.int64, n, 8)
    keys_dev.copy_(torch.from_numpy(first))
    es.sort_noalloc(keys_dev, out=out)  # the device's scratch address is looked up before capture
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        es.sort_noalloc(keys_dev, out=out)
    for seed in (9, 10, 11):
        keys = _keys(np.int64, n, seed)
        keys_dev.copy_(torch.from_numpy(keys))
        graph.replay()
        torch.cuda.synchronize()
        assert_bits_equal(to_np(out), oracle.sort(keys), f"replay {seed}")
        # eager library work between replays
        assert_bits_equal(to_np(es.sort(keys_dev)), oracle.sort(keys), "eager between replays")
