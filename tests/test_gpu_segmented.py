"""GPU parity of the batched segmented sort against the oracle, bit for bit.

A batch is one buffer cut into segments by int64 offsets; each segment must
come out as the stable sort of that segment alone (the oracle sorts them one
by one), and keys outside the segments must be left untouched.  The batches
mix sizes across every one-workgroup class boundary and the long-segment
radix passes (one tile, one tile + 1, several tiles with a ragged end), empty
segments, gaps before and after the segments, every key type, 4- and 8-byte
values, skewed keys, in-place calls, every tunable that may change the route
(the bytes must not change), bad offsets, and replays of a captured HIP graph
with new keys and offsets between replays.
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

DTYPES = [np.uint32, np.int32, np.float32, np.int64, np.float64]
# sizes around every class capacity (512, 2048, 4096, 8192, 16384) and the
# tile sizes of the long-segment passes (8192, 12288 keys)
BOUNDARY_SIZES = [0, 1, 2, 3, 63, 64, 65, 511, 512, 513, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193,
                  12287, 12288, 12289, 16383, 16384, 16385, 24576, 24577, 40_000, 0, 5]


def _batch(seed, extra=200, median=300.0, sigma=1.5, hi=20_000, lead=7, tail=9):
    sizes = np.concatenate([np.array(BOUNDARY_SIZES, dtype=np.int64),
                            workloads.segment_sizes(extra, seed=seed, median=median, sigma=sigma, lo=0, hi=hi)])
    workloads.rng(seed).shuffle(sizes)
    offs = workloads.segment_offsets(sizes) + lead
    n = int(offs[-1]) + tail
    return offs, n


def _keys(dt, n, seed):
    keys = workloads.uniform(dt, n, seed)
    g = np.random.default_rng(seed)
    keys[g.integers(0, n, n // 4)] = keys[g.integers(0, n, n // 4)]  # duplicates: stability is visible
    return keys


def _run_keys(es, keys, offs, params=None, in_place=False):
    import torch

    k = to_dev(keys)
    o = torch.from_numpy(offs).cuda()
    if in_place:
        return to_np(es.segmented_sort(k, o, out=k, params=params))
    out = k.clone()  # positions outside the segments must keep these bytes
    return to_np(es.segmented_sort(k, o, out=out, params=params))


@pytest.mark.parametrize("dt", DTYPES)
def test_segmented_keys(dt):
    es = require_gpu()
    offs, n = _batch(1)
    keys = _keys(dt, n, 2)
    got = _run_keys(es, keys, offs)
    assert_bits_equal(got, oracle.segmented_sort(keys, offs), f"segmented {np.dtype(dt).name}")


@pytest.mark.parametrize("vb", [4, 8])
@pytest.mark.parametrize("dt", DTYPES)
def test_segmented_pairs(dt, vb):
    import torch

    es = require_gpu()
    offs, n = _batch(3)
    keys = _keys(dt, n, 4)
    vals = (np.arange(n, dtype=np.int64) * 2654435761 % (2**61)).astype(np.int64 if vb == 8 else np.int32)
    kd, vd = to_dev(keys), to_dev(vals)
    ko, vo = kd.clone(), vd.clone()
    es.segmented_sort_pairs(kd, vd, torch.from_numpy(offs).cuda(), keys_out=ko, values_out=vo)
    want_k, want_v = oracle.segmented_sort_pairs(keys, vals, offs)
    assert_bits_equal(to_np(ko), want_k, f"segmented pairs keys {np.dtype(dt).name}/{vb}")
    assert_bits_equal(to_np(vo), want_v, f"segmented pairs values {np.dtype(dt).name}/{vb}")


@pytest.mark.parametrize("dist", ["all_equal", "distinct16", "sorted", "reverse", "zipf", "gaussian"])
def test_segmented_distributions(dist):
    es = require_gpu()
    offs, n = _batch(5)
    keys = workloads.make(dist, np.int32, n, 6)
    assert_bits_equal(_run_keys(es, keys, offs), oracle.segmented_sort(keys, offs), f"segmented {dist}")


@pytest.mark.parametrize("dt", [np.uint32, np.float64])
def test_segmented_in_place(dt):
    import torch

    es = require_gpu()
    offs, n = _batch(7, lead=0, tail=0)
    keys = _keys(dt, n, 8)
    assert_bits_equal(_run_keys(es, keys, offs, in_place=True), oracle.segmented_sort(keys, offs), "in place")
    vals = np.arange(n, dtype=np.int32)
    kd, vd = to_dev(keys), to_dev(vals)
    es.segmented_sort_pairs(kd, vd, torch.from_numpy(offs).cuda(), keys_out=kd, values_out=vd)
    want_k, want_v = oracle.segmented_sort_pairs(keys, vals, offs)
    assert_bits_equal(to_np(kd), want_k, "in place pairs keys")
    assert_bits_equal(to_np(vd), want_v, "in place pairs values")


@pytest.mark.parametrize("shape", [(512, 24), (512, 16), (256, 16), (256, 8)])
@pytest.mark.parametrize("fallback", [0, 1, 600, 5000, 1 << 40])
def test_segmented_tunables_do_not_change_bytes(shape, fallback):
    es = require_gpu()
    offs, n = _batch(9)
    keys = _keys(np.uint32, n, 10)
    p = es.default_params(fallback_threshold=fallback, block_threads=shape[0], items_per_thread=shape[1])
    assert_bits_equal(_run_keys(es, keys, offs, p), oracle.segmented_sort(keys, offs),
                      f"fallback {fallback} shape {shape}")


def test_segmented_routes_match_the_size_classes():
    import torch

    es = require_gpu()
    offs, n = _batch(11)
    keys = _keys(np.uint32, n, 12)
    k = to_dev(keys)
    o = torch.from_numpy(offs).cuda()
    p = es.default_params(block_threads=512, items_per_thread=24)  # a known tile size
    tmp = torch.empty(es.segmented_temp_bytes(es.UINT32, n, offs.size - 1, 0, p), dtype=torch.uint8, device="cuda")
    out = es.segmented_sort(k, o, params=p, temp=tmp)
    st = es.segmented_stats(tmp)
    sizes = np.diff(offs)
    caps = [512, 2048, 8192, 16384]
    want = [0, 0, 0, 0]
    for s in sizes[(sizes > 0) & (sizes < 16384)]:
        want[next(c for c in range(4) if s <= caps[c])] += 1
    assert st["block_classes"] == want
    big = sizes[sizes >= 16384]
    assert st["large"] == big.size
    plan_tile = 512 * 24
    assert st["tiles"] == int(np.sum((big + plan_tile - 1) // plan_tile))
    assert es.check_device_error(tmp) == es.OK
    got = to_np(out)
    want_k = oracle.segmented_sort(keys, offs)
    for b, e in zip(offs[:-1], offs[1:]):
        assert_bits_equal(got[b:e], want_k[b:e], "segment")


def test_segmented_many_tiny_segments():
    es = require_gpu()
    sizes = workloads.segment_sizes(20_000, seed=13, median=6, sigma=1.0, lo=0, hi=40)
    offs = workloads.segment_offsets(sizes)
    keys = _keys(np.int64, int(offs[-1]), 14)
    assert_bits_equal(_run_keys(es, keys, offs), oracle.segmented_sort(keys, offs), "tiny segments")


def test_segmented_long_segments_only():
    import torch

    es = require_gpu()
    sizes = np.array([200_000, 100_001, 16385, 12288 * 3, 1], dtype=np.int64)
    offs = workloads.segment_offsets(sizes)
    n = int(offs[-1])
    keys = _keys(np.float64, n, 15)
    vals = np.arange(n, dtype=np.int64)
    p = es.default_params(fallback_threshold=0)
    kd, vd = to_dev(keys), to_dev(vals)
    ko, vo = es.segmented_sort_pairs(kd, vd, torch.from_numpy(offs).cuda(), params=p)
    want_k, want_v = oracle.segmented_sort_pairs(keys, vals, offs)
    assert_bits_equal(to_np(ko), want_k, "long segments keys")
    assert_bits_equal(to_np(vo), want_v, "long segments values")


def test_segmented_empty_batches():
    import torch

    es = require_gpu()
    k = to_dev(np.arange(10, dtype=np.int32)[::-1].copy())
    out = k.clone()
    es.segmented_sort(k, torch.zeros(1, dtype=torch.int64, device="cuda"), out=out)  # no segments
    assert np.array_equal(to_np(out), np.arange(10)[::-1])
    e = to_dev(np.zeros(0, dtype=np.int32))
    es.segmented_sort(e, torch.zeros(4, dtype=torch.int64, device="cuda"))  # three empty segments of nothing


@pytest.mark.parametrize("offs", [[0, 1000, 3000, 2500, 5000],   # decreasing
                                  [0, 1000, 3000, 6000],         # past n
                                  [-1, 1000, 5000],              # before 0
                                  [0, 10, 5, 6, 20]])            # overlapping segments
def test_segmented_bad_offsets_write_nothing(offs):
    import torch

    es = require_gpu()
    n = 5000
    keys = _keys(np.uint32, n, 16)
    offs = np.array(offs, dtype=np.int64)
    k = to_dev(keys)
    out = k.clone()
    tmp = torch.empty(es.segmented_temp_bytes(es.UINT32, n, offs.size - 1), dtype=torch.uint8, device="cuda")
    es.segmented_sort(k, torch.from_numpy(offs).cuda(), out=out, temp=tmp)
    assert es.check_device_error(tmp) == es.ERR_INVALID_ARG
    assert_bits_equal(to_np(out), keys, "nothing written")
    assert es.segmented_stats(tmp)["large"] == 0
    # the error word is cleared by the next good call on the same scratch
    good = np.array([0, 1000, 3000], dtype=np.int64)
    es.segmented_sort(k, torch.from_numpy(good).cuda(), out=out, temp=tmp)
    assert es.check_device_error(tmp) == es.OK
    got = to_np(out)
    assert_bits_equal(got[0:1000], oracle.sort(keys[0:1000]), "first segment")
    assert_bits_equal(got[1000:3000], oracle.sort(keys[1000:3000]), "second segment")


def test_sort_each_matches_oracle():
    es = require_gpu()
    offs, n = _batch(17, extra=40)
    keys = _keys(np.int32, n, 18)
    k = to_dev(keys)
    out = k.clone()
    es.sort_each(k, offs, out=out)
    assert_bits_equal(to_np(out), oracle.segmented_sort(keys, offs), "sort_each keys")
    vals = np.arange(n, dtype=np.int64) * 3
    vd = to_dev(vals)
    ko, vo = k.clone(), vd.clone()
    es.sort_each(k, offs, vd, out=ko, values_out=vo)
    want_k, want_v = oracle.segmented_sort_pairs(keys, vals, offs)
    assert_bits_equal(to_np(ko), want_k, "sort_each pairs keys")
    assert_bits_equal(to_np(vo), want_v, "sort_each pairs values")


def test_segmented_graph_replays_with_new_offsets():
    """One captured graph, replayed with new keys and new offsets (same n and segment count) each time;
    eager library work runs between replays; every replay matches the oracle."""
    import torch

    es = require_gpu()
    nseg = 300
    layouts = []
    for r in range(4):
        sizes = workloads.segment_sizes(nseg, seed=100 + r, median=400, sigma=1.8, lo=0, hi=60_000)
        layouts.append(sizes)
    n = int(max(s.sum() for s in layouts))
    keys_dev = torch.empty(n, dtype=torch.int32, device="cuda")
    offs_dev = torch.empty(nseg + 1, dtype=torch.int64, device="cuda")
    out = torch.empty_like(keys_dev)
    tmp = torch.empty(es.segmented_temp_bytes(es.INT32, n, nseg), dtype=torch.uint8, device="cuda")

    def load(r):
        offs = workloads.segment_offsets(layouts[r])
        keys = _keys(np.int32, n, 200 + r)
        keys_dev.copy_(torch.from_numpy(keys))
        offs_dev.copy_(torch.from_numpy(offs))
        out.copy_(keys_dev)
        return keys, offs

    keys, offs = load(0)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up outside capture
        es.segmented_sort(keys_dev, offs_dev, out=out, temp=tmp)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    assert_bits_equal(to_np(out), oracle.segmented_sort(keys, offs), "eager warm-up")

    graph = torch.cuda.CUDAGraph()
    keys, offs = load(1)
    with torch.cuda.graph(graph):
        es.segmented_sort(keys_dev, offs_dev, out=out, temp=tmp)
    for r in (1, 2, 3, 0):
        keys, offs = load(r)
        graph.replay()
        torch.cuda.synchronize()
        assert es.check_device_error(tmp) == es.OK
        assert_bits_equal(to_np(out), oracle.segmented_sort(keys, offs), f"replay with layout {r}")
        # eager library work between replays
        x = to_dev(workloads.uniform(np.int32, 50_000, r))
        assert oracle.first_unsorted(to_np(es.sort(x))) == -1
