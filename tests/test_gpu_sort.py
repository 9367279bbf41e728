"""GPU parity of the three library sorts against the oracle, bit for bit.

Covers every routine the adaptive partition sort can pick (Sec. 4.3,
Algorithm 6): the one-workgroup small-array sort, the LSD radix sort and the
mergesort; every key type; keys-only, key-value (4- and 8-byte values) and
argsort (int32 and int64 indices); sizes from 0 to several tiles with ragged
ends; float edge values; in-place calls; and the result's independence from
every tunable (the stable sort is unique, so all settings give the same bytes).
"""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, check_sort_full, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

DTYPES = [np.uint32, np.int32, np.float32, np.int64, np.float64]


def _params(es, path):
    if path == "radix":
        return es.default_params(algo=es.ALGO_RADIX, fallback_threshold=0)
    if path == "merge":
        return es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0)
    if path == "small":
        return es.default_params(fallback_threshold=1 << 40)
    return None


@pytest.mark.parametrize("path", ["radix", "merge"])
@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 63, 4096, 4097, 9000, 70_001])
def test_sort_all_ops(path, dt, n):
    es = require_gpu()
    keys = workloads.uniform(dt, n, n + 11)
    g = np.random.default_rng(n)
    if n > 8:  # duplicates, so stability is visible in pairs and argsort
        keys[g.integers(0, n, n // 4)] = keys[g.integers(0, n, n // 4)]
    check_sort_full(es, keys, _params(es, path), f"{path} {np.dtype(dt).name} n={n}")


@pytest.mark.parametrize("dt", DTYPES)
# sizes on both sides of every workgroup shape of the one-workgroup sort
@pytest.mark.parametrize("n", [2, 3, 100, 512, 513, 1000, 1025, 2048, 2049, 4095, 4097, 8191, 8192, 8193, 16383])
def test_small_path(dt, n):
    es = require_gpu()
    cap = es.plan(es.OP_SORT, es.dtype_code(_torch_dtype(dt)), n)["small_capacity"]
    if n > cap:
        pytest.skip("beyond the one-workgroup capacity of this key width")
    p = _params(es, "small")
    assert es.plan(es.OP_SORT, es.dtype_code(_torch_dtype(dt)), n, 0, p)["path_name"] == "small"
    keys = workloads.uniform(dt, n, n)
    keys[::3] = keys[0]
    check_sort_full(es, keys, p, f"small {np.dtype(dt).name} n={n}")


def test_small_path_at_capacity():
    es = require_gpu()
    import torch

    for dt, tdt in ((np.uint32, torch.uint32), (np.int64, torch.int64)):
        cap = es.plan(es.OP_SORT, es.dtype_code(tdt), 10)["small_capacity"]
        p = es.default_params(fallback_threshold=cap + 1)
        assert es.plan(es.OP_SORT, es.dtype_code(tdt), cap, 0, p)["path_name"] == "small"
        keys = workloads.uniform(dt, cap, 5)
        check_sort_full(es, keys, p, f"small capacity {cap}")


def _torch_dtype(dt):
    import torch

    return {np.uint32: torch.uint32, np.int32: torch.int32, np.float32: torch.float32, np.int64: torch.int64,
            np.float64: torch.float64}[dt]


@pytest.mark.parametrize("path", ["small", "radix", "merge"])
@pytest.mark.parametrize("dt", [np.float32, np.float64])
def test_float_edge_values(path, dt):
    es = require_gpu()
    g = np.random.default_rng(1)
    edges = workloads.float_edges(dt)
    nan_bits = {np.float32: [0x7FC00000, 0xFFC00000, 0x7F800001], np.float64: [0x7FF8000000000000,
                                                                                   0xFFF8000000000000]}[dt]
    nans = np.array(nan_bits, dtype=np.uint32 if dt == np.float32 else np.uint64).view(dt)
    pool = np.concatenate([edges, nans])
    keys = pool[g.integers(0, pool.size, 5000)]
    check_sort_full(es, keys, _params(es, path), f"float edges {path}")


@pytest.mark.parametrize("path", ["radix", "merge", "small"])
@pytest.mark.parametrize("dist", ["sorted", "reverse", "nearly_sorted", "distinct16", "zipf", "all_equal",
                                  "gaussian"])
def test_distributions(path, dist):
    es = require_gpu()
    n = 12_000 if path == "small" else 50_000
    keys = workloads.make(dist, np.int32, n, 3)
    check_sort_full(es, keys, _params(es, path), f"{dist} {path}")


def test_config0_uint32_1e6_default_params():
    """1e6 uint32 keys, uniform over [0, 2^32), seed 42, 8-bit digits, untuned defaults."""
    es = require_gpu()
    keys = workloads.uniform(np.uint32, 1_000_000, workloads.DEFAULT_SEED)
    info = es.plan(es.OP_SORT, es.UINT32, keys.size)
    assert info["path_name"] == "radix" and info["passes"] == 4
    got = to_np(es.sort(to_dev(keys)))
    assert_bits_equal(got, oracle.sort(keys), "config 0")


@pytest.mark.parametrize("bits", [4, 5, 6, 7, 8, 9, 10, 11, 12])
def test_digit_width_invariance(bits):
    es = require_gpu()
    keys = workloads.uniform(np.int64, 33_333, bits)
    keys[::5] = keys[7]
    want_perm = oracle.stable_perm(keys)
    p = es.default_params(digit_bits=bits, fallback_threshold=0)
    assert_bits_equal(to_np(es.sort(to_dev(keys), params=p)), keys[want_perm], f"bits {bits}")
    assert np.array_equal(to_np(es.argsort(to_dev(keys), params=p)), want_perm)
    k32 = workloads.uniform(np.float32, 33_333, bits)
    assert_bits_equal(to_np(es.sort(to_dev(k32), params=p)), oracle.sort(k32), f"bits {bits} f32")


@pytest.mark.parametrize("t_ins", [1, 2, 3, 17, 64, 195, 629, 2048])
def test_insertion_threshold_invariance(t_ins):
    es = require_gpu()
    for dt in (np.int32, np.float64):
        keys = workloads.uniform(dt, 40_000 + t_ins, t_ins)
        keys[::4] = keys[1]
        p = es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0, insertion_threshold=t_ins)
        perm = oracle.stable_perm(keys)
        assert_bits_equal(to_np(es.sort(to_dev(keys), params=p)), keys[perm], f"T_ins {t_ins}")
        assert np.array_equal(to_np(es.argsort(to_dev(keys), params=p)), perm)


@pytest.mark.parametrize("shape", [(256, 8), (256, 12), (256, 24), (256, 32), (512, 8), (512, 16)])
def test_tile_shape_invariance(shape):
    es = require_gpu()
    keys = workloads.uniform(np.int32, 200_001, shape[1])
    p = es.default_params(block_threads=shape[0], items_per_thread=shape[1], fallback_threshold=0)
    assert_bits_equal(to_np(es.sort(to_dev(keys), params=p)), oracle.sort(keys), f"shape {shape}")


@pytest.mark.parametrize("path", ["small", "radix", "merge"])
@pytest.mark.parametrize("dt", [np.int32, np.float64])
def test_in_place(path, dt):
    es = require_gpu()
    n = 5000 if path == "small" else 60_000
    keys = workloads.uniform(dt, n, 9)
    keys[::2] = keys[3]
    vals = np.arange(n, dtype=np.int64)
    perm = oracle.stable_perm(keys)
    p = _params(es, path)
    for bits in ([8, 11] if path == "radix" else [8]):  # 11 bits: odd pass count on 32-bit keys
        if path == "radix":
            p = es.default_params(algo=es.ALGO_RADIX, fallback_threshold=0, digit_bits=bits)
        k = to_dev(keys)
        es.sort(k, out=k, params=p)
        assert_bits_equal(to_np(k), keys[perm], f"in-place sort {path} bits {bits}")
        k = to_dev(keys)
        v = to_dev(vals)
        es.sort_pairs(k, v, keys_out=k, values_out=v, params=p)
        assert_bits_equal(to_np(k), keys[perm], f"in-place pairs keys {path}")
        assert_bits_equal(to_np(v), vals[perm], f"in-place pairs values {path}")


def test_repeat_is_deterministic():
    es = require_gpu()
    keys = workloads.uniform(np.uint32, 300_000, 77)
    k = to_dev(keys)
    first = to_np(es.argsort(k))
    for _ in range(20):
        assert np.array_equal(to_np(es.argsort(k)), first)
    assert np.array_equal(first, oracle.stable_perm(keys))


def test_lookback_timeout_is_reported_not_hung():
    """Tile 0 withholds its counts: the bounded look-back wait runs out and is reported -- by the next
    library call once the failing kernel has run, by the check on its scratch, and at once in checked mode.
    Each failure is reported once; afterwards the library sorts normally."""
    es = require_gpu()
    import torch

    keys = workloads.uniform(np.uint32, 50_000, 1)
    k = to_dev(keys)
    bad = es.default_params(fallback_threshold=0, spin_limit=2000, debug_flags=es.DEBUG_WITHHOLD_TILE0)
    good = es.default_params(fallback_threshold=0)
    need = es.temp_bytes(es.OP_SORT, es.UINT32, keys.size, 0, bad)
    temp = torch.empty(need, dtype=torch.uint8, device="cuda")
    # 1. the failing call returns (its kernels run later); the next call reports it and enqueues nothing
    es.sort(k, params=bad, temp=temp)
    torch.cuda.synchronize()
    out = torch.zeros_like(k)
    with pytest.raises(es.EvosortError) as e:
        es.sort(k, params=good, out=out)
    assert e.value.status == es.ERR_DEVICE_TIMEOUT
    torch.cuda.synchronize()
    assert not bool(out.view(torch.int32).any().item()), "the reporting call enqueued nothing"
    assert es.check_device_error(temp) == es.ERR_DEVICE_TIMEOUT  # still recorded in the failed call's scratch
    # 2. reported once: the next call runs
    assert_bits_equal(to_np(es.sort(k, params=good)), oracle.sort(keys), "after the report")
    # 3. checked mode raises from the failing call itself, and the failure is not reported again
    with pytest.raises(es.EvosortError) as e:
        es.sort(k, params=bad, temp=temp, check=True)
    assert e.value.status == es.ERR_DEVICE_TIMEOUT
    for op in ("pairs", "argsort"):
        with pytest.raises(es.EvosortError) as e:
            if op == "pairs":
                es.sort_pairs(k, k.view(torch.int32).clone(), params=bad, check=True)
            else:
                es.argsort(k, params=bad, check=True)
        assert e.value.status == es.ERR_DEVICE_TIMEOUT, op
    # 4. the same scratch, used normally afterwards, reports no error and sorts right
    out = es.sort(k, params=good, temp=temp, check=True)
    assert es.check_device_error(temp) == es.OK
    assert_bits_equal(to_np(out), oracle.sort(keys), "after timeout")


def test_error_word_is_cleared_by_every_routine():
    """A scratch buffer whose error word was set by a failed radix call reads clear after a small-array,
    mergesort or radix call reuses it."""
    es = require_gpu()
    import torch

    keys = workloads.uniform(np.int32, 40_000, 2)
    k = to_dev(keys)
    bad = es.default_params(fallback_threshold=0, spin_limit=2000, debug_flags=es.DEBUG_WITHHOLD_TILE0)
    temp = torch.empty(es.temp_bytes(es.OP_SORT, es.INT32, keys.size, 0, bad), dtype=torch.uint8, device="cuda")
    for path, params, n in (("small", es.default_params(), 3000),
                            ("merge", es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0), keys.size),
                            ("radix", es.default_params(fallback_threshold=0), keys.size)):
        with pytest.raises(es.EvosortError):
            es.sort(k, params=bad, temp=temp, check=True)
        assert es.check_device_error(temp) == es.ERR_DEVICE_TIMEOUT
        assert es.plan(es.OP_SORT, es.INT32, n, 0, params)["path_name"] == path
        out = es.sort(k[:n], params=params, temp=temp, check=True)
        assert es.check_device_error(temp) == es.OK, path
        assert_bits_equal(to_np(out), oracle.sort(keys[:n]), path)


def test_call_on_a_side_stream_keeps_its_buffers():
    """A sort enqueued on another stream than the current one: the scratch and output the binding
    allocates are held for that stream, so allocations and writes on the current stream right after the
    call cannot land in them while the sort still runs."""
    es = require_gpu()
    import torch

    n = 1 << 24
    keys = workloads.uniform(np.int32, n, 5)
    k = to_dev(keys)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    results = []
    for _ in range(3):
        results.append(es.sort(k, stream=side))          # binding-allocated scratch, freed on return
        junk = torch.empty(3 * n, dtype=torch.int32, device="cuda")
        junk.fill_(-1)                                   # current stream: must not reuse that memory yet
        del junk
    side.synchronize()
    want = oracle.sort(keys)
    for r in results:
        assert_bits_equal(to_np(r), want, "side-stream sort")


@pytest.mark.parametrize("path", ["small", "radix", "merge"])
@pytest.mark.parametrize("op", ["keys", "pairs", "argsort"])
def test_graph_capture_replays_with_new_inputs(path, op):
    """One sort captured in a HIP graph (through torch.cuda.graph) and replayed with new contents in the
    captured input buffers; eager library work runs between replays; every replay matches the oracle.
    The launch sequence has no memset and no host synchronisation, so capture is allowed."""
    import torch

    es = require_gpu()
    n = 12_000 if path == "small" else 150_001
    p = _params(es, path)
    keys_dev = torch.empty(n, dtype=torch.int32, device="cuda")
    vals_dev = torch.empty(n, dtype=torch.int64, device="cuda")
    out_k = torch.empty_like(keys_dev)
    out_v = torch.empty_like(vals_dev)
    code = es.dtype_code(keys_dev.dtype)
    opc = {"keys": es.OP_SORT, "pairs": es.OP_SORT_PAIRS, "argsort": es.OP_ARGSORT}[op]
    vbytes = 8 if op != "keys" else 0
    assert es.plan(opc, code, n, vbytes, p)["path_name"] == path
    tmp = torch.empty(max(es.temp_bytes(opc, code, n, vbytes, p), 256), dtype=torch.uint8, device="cuda")

    def call():
        if op == "keys":
            es.sort(keys_dev, params=p, out=out_k, temp=tmp)
        elif op == "pairs":
            es.sort_pairs(keys_dev, vals_dev, params=p, keys_out=out_k, values_out=out_v, temp=tmp)
        else:
            es.argsort(keys_dev, index_dtype=torch.int64, params=p, out=out_v, temp=tmp)

    def load(r):
        keys = workloads.uniform(np.int32, n, 300 + r)
        keys[::7] = keys[1]  # ties
        vals = (np.arange(n, dtype=np.int64) * 7919 + r).astype(np.int64)
        keys_dev.copy_(torch.from_numpy(keys))
        vals_dev.copy_(torch.from_numpy(vals))
        out_k.zero_()
        out_v.zero_()
        return keys, vals

    def check(keys, vals, label):
        perm = oracle.stable_perm(keys)
        if op in ("keys", "pairs"):
            assert_bits_equal(to_np(out_k), keys[perm], f"{label} keys")
        if op == "pairs":
            assert np.array_equal(to_np(out_v), vals[perm]), f"{label} values"
        if op == "argsort":
            assert np.array_equal(to_np(out_v), perm), f"{label} indices"

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    keys, vals = load(0)
    with torch.cuda.stream(side):  # warm-up outside capture
        call()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    check(keys, vals, "eager")
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()
    for r in (1, 2, 3):
        keys, vals = load(r)
        graph.replay()
        torch.cuda.synchronize()
        if path == "radix":  # the radix path's scratch holds a device error word
            assert es.check_device_error(tmp) == es.OK
        check(keys, vals, f"{path} {op} replay {r}")
        x = to_dev(workloads.uniform(np.int32, 40_000, r))  # eager library work between replays
        assert oracle.first_unsorted(to_np(es.sort(x))) == -1


@pytest.mark.parametrize("dt", [np.int32, np.float64])
def test_pass0_from_tile_prefixes(dt):
    """From 256 tiles on, pass 0 takes its offsets from a scan of the histogram's per-tile counts instead of
    the look-back; small tiles reach that count at a test size (below it the look-back serves pass 0)."""
    import torch

    es = require_gpu()
    p = es.default_params(algo=es.ALGO_RADIX, fallback_threshold=0, block_threads=256, items_per_thread=8)
    tdt = torch.int32 if dt == np.int32 else torch.float64
    for n in (300_001, 2048 * 256 - 1):  # 147 tiles (look-back), 256 tiles (tile prefixes)
        assert es.plan(es.OP_SORT, es.dtype_code(tdt), n, 0, p)["tiles"] == (n + 2047) // 2048
        keys = workloads.float_mix(dt, n, 12) if dt == np.float64 else workloads.uniform(dt, n, 12)
        keys[::5] = keys[3]
        check_sort_full(es, keys, p, f"tile prefixes {np.dtype(dt).name} n={n}")
