"""Radix passes whose digit is the same for every key are skipped on the device (Sec. 4, Algorithm 4's
pass loop: a pass over a constant digit leaves the order unchanged).

The launch sequence is fixed; each pass reads the scan's per-pass flags and either leaves at once or
picks its input and output so that the last live pass writes the output.  Every skip pattern is checked
element by element against the oracle: no live pass (all keys equal: a copy, or the identity permutation),
one, two (adjacent and apart), three and four live passes of 32-bit keys, four of eight for 64-bit keys,
sorted out of place and in place (odd live counts in place end with a copy), keys only, pairs with 4- and
8-byte values, argsort with int32 and int64 indices, ascending and descending, and inside a graph replayed
with inputs whose live passes differ from the captured call's.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

N = 100_003


def _pattern(name, n, seed):
    g = np.random.default_rng(seed)
    r32 = g.integers(0, 2**32, n, dtype=np.uint64)
    if name == "none":              # every key equal: no live pass
        return np.full(n, -12345, dtype=np.int32)
    if name == "byte2":             # one live pass (pass 2)
        return ((r32 & 0xFF) << 16).astype(np.int32)
    if name == "low16":             # two adjacent live passes (0, 1)
        return (r32 & 0xFFF0).astype(np.int32) + 7
    if name == "bytes0and3":        # two live passes apart (0, 3)
        v = ((r32 & 0xFF) | ((r32 >> 8 & 0x3) << 24)).astype(np.uint32)
        return v.view(np.int32)
    if name == "low24":             # three live passes (0, 1, 2)
        return (r32 & 0xFFFFFF).astype(np.int32) + 5
    if name == "zipf":              # ranks < 2^20: three live passes
        return workloads.zipf(np.int32, n, seed)
    if name == "full32":            # four live passes
        return workloads.uniform(np.int32, n, seed)
    if name == "int64_low32":       # 64-bit keys, four live passes of eight
        return (r32 & 0x7FFFFFFF).astype(np.int64) + 12345
    if name == "int64_byte5":       # 64-bit keys, one live pass of eight
        return ((r32 & 0xFF).astype(np.int64) << 40) + 7
    raise ValueError(name)


PATTERNS = ["none", "byte2", "low16", "bytes0and3", "low24", "zipf", "full32", "int64_low32", "int64_byte5"]


def _live_passes(keys):
    """Passes whose 8-bit digit of the order word takes more than one value (from the oracle's order map)."""
    u = oracle.order_keys(keys)
    return [p for p in range(keys.dtype.itemsize) if np.unique((u >> np.uint64(8 * p)) & np.uint64(0xFF)).size > 1]


@pytest.mark.parametrize("desc", [0, 1])
@pytest.mark.parametrize("name", PATTERNS)
def test_skip_patterns(name, desc):
    import torch

    es = require_gpu()
    keys = _pattern(name, N, 3)
    if name != "none":
        keys[::9] = keys[4]  # ties
    live = _live_passes(keys)
    expect_live = {"none": 0, "byte2": 1, "low16": 2, "bytes0and3": 2, "low24": 3, "zipf": 3, "full32": 4,
                   "int64_low32": 4, "int64_byte5": 1}[name]
    assert len(live) == expect_live, live
    p = es.default_params(algo=es.ALGO_RADIX, fallback_threshold=0, descending=desc)
    perm = oracle.stable_perm(keys, descending=bool(desc))
    want = keys[perm]
    k = to_dev(keys)
    assert es.plan(es.OP_SORT, es.dtype_code(k.dtype), N, 0, p)["path_name"] == "radix"
    assert_bits_equal(to_np(es.sort(k, params=p, check=True)), want, "keys")
    v4 = (np.arange(N, dtype=np.int64) * 7 + 1).astype(np.int32)
    v8 = np.arange(N, dtype=np.int64) * 3 - 5
    for vals in (v4, v8):
        ko, vo = es.sort_pairs(k, to_dev(vals), params=p, check=True)
        assert_bits_equal(to_np(ko), want, f"pairs({vals.itemsize}) keys")
        assert_bits_equal(to_np(vo), vals[perm], f"pairs({vals.itemsize}) values")
    for idt in (torch.int32, torch.int64):
        assert np.array_equal(to_np(es.argsort(k, index_dtype=idt, params=p, check=True)), perm), f"argsort {idt}"
    # in place: keys, and pairs with both in place
    kin = to_dev(keys)
    es.sort(kin, params=p, out=kin, check=True)
    assert_bits_equal(to_np(kin), want, "keys in place")
    kin, vin = to_dev(keys), to_dev(v8)
    es.sort_pairs(kin, vin, params=p, keys_out=kin, values_out=vin, check=True)
    assert_bits_equal(to_np(kin), want, "pairs in place keys")
    assert_bits_equal(to_np(vin), v8[perm], "pairs in place values")
    # values in place only
    vin = to_dev(v4)
    ko, _ = es.sort_pairs(k, vin, params=p, values_out=vin, check=True)
    assert_bits_equal(to_np(ko), want, "values in place: keys")
    assert_bits_equal(to_np(vin), v4[perm], "values in place: values")


@pytest.mark.parametrize("name", ["none", "byte2", "low24"])
def test_skip_patterns_with_tile_prefix_route(name):
    """Large enough for pass 0 to take its tile offsets from the histogram (256 tiles and more)."""
    import torch

    es = require_gpu()
    n = 9_000_001
    keys = _pattern(name, n, 4)
    p = es.default_params()
    assert es.plan(es.OP_SORT, es.INT32, n, 0, p)["tiles"] >= 256
    perm = oracle.stable_perm(keys)
    k = to_dev(keys)
    assert_bits_equal(to_np(es.sort(k, params=p, check=True)), keys[perm], "keys")
    assert np.array_equal(to_np(es.argsort(k, index_dtype=torch.int32, params=p, check=True)), perm), "argsort"
    es.sort(k, params=p, out=k, check=True)
    assert_bits_equal(to_np(k), keys[perm], "in place")


def test_graph_replay_with_other_live_passes():
    """The launch sequence does not depend on which passes are live: one captured graph sorts inputs with
    0, 1, 3 and 4 live passes."""
    import torch

    es = require_gpu()
    n = 60_001
    p = es.default_params(fallback_threshold=0)
    keys_dev = torch.empty(n, dtype=torch.int32, device="cuda")
    out = torch.empty_like(keys_dev)
    tmp = torch.empty(es.temp_bytes(es.OP_SORT, es.INT32, n, 0, p), dtype=torch.uint8, device="cuda")
    keys_dev.copy_(torch.from_numpy(_pattern("full32", n, 1)))
    es.sort(keys_dev, params=p, out=out, temp=tmp)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        es.sort(keys_dev, params=p, out=out, temp=tmp)
    for name in ("none", "byte2", "low24", "full32", "none"):
        keys = _pattern(name, n, 2)
        keys_dev.copy_(torch.from_numpy(keys))
        graph.replay()
        torch.cuda.synchronize()
        assert_bits_equal(to_np(out), oracle.sort(keys), f"replay {name}")


def test_stream_copy_and_read():
    import torch

    es = require_gpu()
    for nbytes in (4, 20, 4096 + 12, (1 << 24) + 36):
        src = torch.randint(-2**31, 2**31 - 1, (nbytes // 4,), dtype=torch.int32, device="cuda")
        dst = torch.zeros_like(src)
        es.stream_copy(dst, src)
        torch.cuda.synchronize()
        assert torch.equal(dst, src), nbytes
    # misaligned views take the word-by-word route
    src = torch.randint(-2**31, 2**31 - 1, (100_001,), dtype=torch.int32, device="cuda")
    dst = torch.zeros_like(src)
    es.stream_copy(dst[1:], src[:-1])
    torch.cuda.synchronize()
    assert torch.equal(dst[1:], src[:-1]) and int(dst[0].item()) == 0
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    es.stream_read(src[:100_000], sink)
    torch.cuda.synchronize()
