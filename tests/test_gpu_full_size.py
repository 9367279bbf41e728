"""GPU parity at full benchmark sizes, in the launch configuration the benchmark times.

At these sizes the oracle cannot sort the whole array in test time, so each
result is checked by (1) outputs the oracle computes one by one -- the rank of
sampled input elements under the stable sort -- and (2) properties that
together equal "is the stable sort":

* keys-only: ordered, and the same multiset -- the argsort of the same input
  is a permutation and gathers exactly the sorted keys, or (1e10 keys) a count
  table over all 2^32 values, +1 for every input key and -1 for every output
  key, is zero everywhere;
* argsort / key-value with the original index as value: the indices form a
  permutation, gathering the input by them gives the sorted keys bit for bit,
  and (order key, index) is strictly increasing (stability).

Property checks run on the host with numpy over the copied-back arrays, or on
the GPU with plain torch operations (never with this library).  Workloads:

* 1e9 uniform int32 keys, default parameters (the benchmark's sort);
* 1e9 uniform int64 keys, default parameters (the benchmark's int64 sort),
  keys only and argsort;
* 1e8 int32 keys for each of the eight distributions of the sweep;
* 2^30 - 1 and 2^30 int32 keys, either side of the switch from 32-bit to
  64-bit look-back words;
* 1e8 int32 keys of each of the paper's nine distributions, descending;
* 1e10 uniform int32 keys (about 130 GB of HBM);
* 2e9 float64 keys, N(0,1) with 1 % from {-inf, +inf, -0.0, +0.0}, sorted as
  pairs with an int32 payload equal to the original index.
"""
import os
import sys

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import require_gpu, to_dev, to_np

pytestmark = [pytest.mark.gpu, pytest.mark.full_size]


def _progress(msg):
    sys.stderr.write(f"[full-size] {msg}\n")
    sys.stderr.flush()


def _check_ranks(keys, out, samples, seed):
    """out[rank(i)] == keys[i] for sampled inputs i, rank from the oracle (O(n) each)."""
    g = np.random.default_rng(seed)
    bits = {4: np.uint32, 8: np.uint64}[keys.dtype.itemsize]
    kb, ob = keys.view(bits), out.view(bits)
    for i in g.integers(0, keys.size, samples):
        r = oracle.rank_of(keys, int(i))
        assert ob[r] == kb[i], f"sample {i}: rank {r}"


def _check_argsort_exact(keys, sorted_keys, idx):
    """idx is the stable sorting permutation of keys (sorted_keys computed by the GPU sort)."""
    n = keys.size
    seen = np.zeros(n, dtype=bool)
    seen[idx] = True
    assert seen.all(), "indices are not a permutation"
    del seen
    gathered = keys[idx]
    bits = {4: np.uint32, 8: np.uint64}[keys.dtype.itemsize]
    assert np.array_equal(gathered.view(bits), sorted_keys.view(bits)), "gather by indices differs from sorted keys"
    del gathered
    assert oracle.first_unsorted(sorted_keys) == -1, "sorted keys out of order"
    same = sorted_keys.view(bits)[1:] == sorted_keys.view(bits)[:-1]
    assert np.all(idx[1:][same] > idx[:-1][same]), "equal keys not in input order"


@pytest.mark.timeout(900)
def test_benchmark_sort_1e9_int32():
    es = require_gpu()
    import torch

    n = 1_000_000_000
    _progress("1e9 int32: generating")
    keys = workloads.uniform(np.int32, n, workloads.DEFAULT_SEED)
    d_keys = to_dev(keys)
    info = es.plan(es.OP_SORT, es.INT32, n)
    assert info["path_name"] == "radix"
    _progress("1e9 int32: sorting")
    out = to_np(es.sort(d_keys))
    idx = to_np(es.argsort(d_keys, index_dtype=torch.int32)).astype(np.int64)
    del d_keys
    torch.cuda.empty_cache()
    _progress("1e9 int32: oracle samples")
    _check_ranks(keys, out, 6, 1)
    _progress("1e9 int32: exact properties")
    _check_argsort_exact(keys, out, idx)


@pytest.mark.timeout(900)
def test_benchmark_sort_1e9_int64():
    """The 1e9 int64 sort the benchmark times (768 x 12 tiles, eight passes), keys only and argsort with
    int32 indices (512 x 24 tiles of 8-byte keys and 4-byte values)."""
    es = require_gpu()
    import torch

    n = 1_000_000_000
    _progress("1e9 int64: generating")
    keys = workloads.uniform(np.int64, n, workloads.DEFAULT_SEED + 1)
    keys[: n // 4] = keys[n // 4: n // 2]  # a quarter of the keys appear twice: ties
    d_keys = to_dev(keys)
    info = es.plan(es.OP_SORT, es.INT64, n)
    assert info["path_name"] == "radix" and (info["block_threads"], info["items_per_thread"]) == (768, 12)
    _progress("1e9 int64: sorting")
    out = to_np(es.sort(d_keys, check=True))
    idx = to_np(es.argsort(d_keys, index_dtype=torch.int32, check=True)).astype(np.int64)
    del d_keys
    torch.cuda.empty_cache()
    _progress("1e9 int64: oracle samples")
    _check_ranks(keys, out, 4, 8)
    _progress("1e9 int64: exact properties")
    _check_argsort_exact(keys, out, idx)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dist", workloads.DISTRIBUTIONS)
def test_distribution_sweep_1e8_int32(dist):
    es = require_gpu()
    n = 100_000_000
    keys = workloads.make(dist, np.int32, n, 42 + workloads.DISTRIBUTIONS.index(dist))
    d_keys = to_dev(keys)
    out = to_np(es.sort(d_keys))
    idx = to_np(es.argsort(d_keys))
    _check_ranks(keys, out, 4, 2)
    _check_argsort_exact(keys, out, idx)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dist", ["uniform", "distinct16"])
def test_merge_routine_1e8_int32(dist):
    es = require_gpu()
    n = 100_000_000
    keys = workloads.make(dist, np.int32, n, 7)
    d_keys = to_dev(keys)
    p = es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0)
    out = to_np(es.sort(d_keys, params=p))
    idx = to_np(es.argsort(d_keys, params=p))
    _check_ranks(keys, out, 3, 3)
    _check_argsort_exact(keys, out, idx)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("n", [2**30 - 1, 2**30])
def test_lookback_word_width_boundary_int32(n):
    """The largest sort with 32-bit look-back words (n = 2^30 - 1: counts up to 2^30 - 1 in 30 bits) and
    the smallest with 64-bit words (n = 2^30)."""
    es = require_gpu()
    import torch

    info = es.plan(es.OP_SORT, es.INT32, n)
    assert info["path_name"] == "radix" and info["status_bytes"] == (4 if n < 2**30 else 8)
    _progress(f"{n} int32: generating")
    keys = workloads.uniform(np.int32, n, 11)
    keys[: n // 3] = keys[n // 3: 2 * (n // 3)]  # every key of the first third appears twice: ties
    d_keys = to_dev(keys)
    _progress(f"{n} int32: sorting")
    out = to_np(es.sort(d_keys))
    idx = to_np(es.argsort(d_keys, index_dtype=torch.int32)).astype(np.int64)
    del d_keys
    torch.cuda.empty_cache()
    _progress(f"{n} int32: oracle samples")
    _check_ranks(keys, out, 4, 6)
    _progress(f"{n} int32: exact properties")
    _check_argsort_exact(keys, out, idx)


@pytest.mark.timeout(900)
@pytest.mark.parametrize("dist", workloads.PAPER_DISTRIBUTIONS)
def test_paper_distributions_1e8_int32_descending(dist):
    """The paper's nine distributions at 1e8, descending.  For int32, bitwise NOT reverses the order
    (~k = -k - 1), so the stable descending sort of k is the stable ascending sort of ~k: oracle ranks and
    the exact properties are taken on ~k."""
    es = require_gpu()
    n = 100_000_000
    keys = workloads.make(dist, np.int32, n, 42)
    d_keys = to_dev(keys)
    p = es.default_params(descending=1)
    out = to_np(es.sort(d_keys, params=p))
    idx = to_np(es.argsort(d_keys, params=p))
    comp = np.invert(keys)
    _check_ranks(comp, np.invert(out), 4, 7)
    _check_argsort_exact(comp, np.invert(out), idx)


def _gpu_sorted_int(t):
    return bool((t[1:] >= t[:-1]).all().item())


@pytest.mark.timeout(1200)
def test_1e10_int32_keys():
    es = require_gpu()
    import torch

    n = 10_000_000_000
    free, _ = torch.cuda.mem_get_info()
    if free < 140 * 2**30:
        pytest.skip("needs about 140 GB of free HBM")
    _progress("1e10 int32: generating")
    keys = workloads.uniform(np.int32, n, workloads.DEFAULT_SEED)
    d_keys = torch.empty(n, dtype=torch.int32, device="cuda")
    step = 1 << 30
    for s in range(0, n, step):
        d_keys[s:s + step].copy_(torch.from_numpy(keys[s:s + step]))
    info = es.plan(es.OP_SORT, es.INT32, n)
    assert info["path_name"] == "radix" and info["status_bytes"] == 8
    _progress("1e10 int32: sorting")
    d_temp_holder = torch.empty(es.temp_bytes(es.OP_SORT, es.INT32, n), dtype=torch.uint8, device="cuda")
    d_out = es.sort(d_keys, temp=d_temp_holder, check=True)
    del d_temp_holder
    torch.cuda.empty_cache()
    _progress("1e10 int32: properties on the GPU")
    # ordered
    for s in range(0, n - 1, step):
        e = min(s + step + 1, n)
        assert _gpu_sorted_int(d_out[s:e]), f"out of order in [{s}, {e})"
    # same multiset, exactly: one int32 counter per 32-bit value (16 GiB), +1 for every input key and -1
    # for every output key; all counters must end at zero.  Together with the order this is equality with
    # the sorted input, which is unique for keys only.
    counts = torch.zeros(1 << 32, dtype=torch.int32, device="cuda")
    for src, sign in ((d_keys, 1), (d_out, -1)):
        delta = torch.full((step,), sign, dtype=torch.int32, device="cuda")
        for s in range(0, n, step):
            chunk = src[s:s + step]
            slot = chunk.to(torch.int64) + 2**31  # the key's offset-binary value, 0 .. 2^32 - 1
            counts.index_add_(0, slot, delta[:chunk.numel()])
            del slot
        del delta
    assert not bool(counts.any().item()), "the output is not a permutation of the input"
    del counts
    torch.cuda.empty_cache()
    _progress("1e10 int32: oracle samples")
    out_host = np.empty(n, dtype=np.int32)
    for s in range(0, n, step):
        out_host[s:s + step] = d_out[s:s + step].cpu().numpy()
    _check_ranks(keys, out_host, 2, 4)


@pytest.mark.timeout(1200)
def test_2e9_float64_pairs_with_index_payload():
    es = require_gpu()
    import torch

    n = 2_000_000_000
    free, _ = torch.cuda.mem_get_info()
    if free < 90 * 2**30:
        pytest.skip("needs about 90 GB of free HBM")
    _progress("2e9 float64 pairs: generating")
    keys = workloads.float_mix(np.float64, n, workloads.DEFAULT_SEED)
    d_keys = torch.from_numpy(keys).cuda()
    d_vals = torch.arange(n, dtype=torch.int32, device="cuda")
    _progress("2e9 float64 pairs: sorting")
    k_out, v_out = es.sort_pairs(d_keys, d_vals)
    torch.cuda.synchronize()
    del d_vals
    _progress("2e9 float64 pairs: properties on the GPU")
    step = 1 << 28
    # values are a permutation of 0..n-1
    seen = torch.zeros(n, dtype=torch.bool, device="cuda")
    seen[v_out.to(torch.int64)] = True
    assert bool(seen.all().item()), "payload is not a permutation"
    del seen
    # keys_out[j] has the bits of keys_in[v_out[j]]
    kin_bits = d_keys.view(torch.int64)
    kout_bits = k_out.view(torch.int64)
    for s in range(0, n, step):
        idx = v_out[s:s + step].to(torch.int64)
        assert torch.equal(kin_bits[idx], kout_bits[s:s + step]), f"gathered keys differ in [{s}, {s + step})"
    # (order key, index) strictly increasing: order key of a float64 bit
    # pattern b is b with the sign bit flipped when b >= 0, else ~b; compare
    # as signed after flipping the sign bit once more, i.e. b ^ (b>>63 & 0x7fff...) for b < 0
    mag = torch.tensor(0x7FFFFFFFFFFFFFFF, dtype=torch.int64, device="cuda")
    for s in range(0, n - 1, step):
        e = min(s + step + 1, n)
        b = kout_bits[s:e]
        key = torch.where(b < 0, b ^ mag, b)  # signed total order of the float bit patterns
        v = v_out[s:e]
        ok = (key[1:] > key[:-1]) | ((key[1:] == key[:-1]) & (v[1:] > v[:-1]))
        assert bool(ok.all().item()), f"not strictly increasing in [{s}, {e})"
    _progress("2e9 float64 pairs: oracle samples")
    out_host = k_out[: n].cpu().numpy()
    _check_ranks(keys, out_host, 2, 5)
