"""Helpers for the GPU parity tests: device transfer, oracle comparison."""
from __future__ import annotations

import numpy as np
import pytest

import oracle

NP_TO_TORCH = None


def torch_mod():
    import torch

    return torch


def require_gpu():
    """GPU tests fail loudly (not skip) when there is no GPU or no built library."""
    torch = torch_mod()
    if not torch.cuda.is_available():
        pytest.fail("GPU test run without a visible GPU")
    import paper_2505_18681_amd as es  # raises ImportError if the library is missing

    return es


def to_dev(a: np.ndarray):
    torch = torch_mod()
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        return torch.from_numpy(a.view(np.int32)).cuda().view(torch.uint32)
    if a.dtype == np.uint64:
        return torch.from_numpy(a.view(np.int64)).cuda()
    return torch.from_numpy(a).cuda()


def to_np(t, dtype=None) -> np.ndarray:
    torch = torch_mod()
    torch.cuda.synchronize()
    if t.dtype == getattr(torch, "uint32", None):
        return t.view(torch.int32).cpu().numpy().view(np.uint32)
    a = t.cpu().numpy()
    return a.view(dtype) if dtype is not None else a


def bits_view(a: np.ndarray) -> np.ndarray:
    """Bit patterns (so -0.0 vs +0.0 and NaN payloads compare exactly)."""
    return a.view({4: np.uint32, 8: np.uint64}[a.dtype.itemsize])


def assert_bits_equal(got: np.ndarray, want: np.ndarray, what: str):
    g, w = bits_view(np.ascontiguousarray(got)), bits_view(np.ascontiguousarray(want))
    assert g.shape == w.shape, f"{what}: shape {g.shape} != {w.shape}"
    bad = np.flatnonzero(g != w)
    assert bad.size == 0, (f"{what}: {bad.size} of {g.size} elements differ; first at {bad[0]}: "
                           f"got {got[bad[0]]!r} want {want[bad[0]]!r}")


def check_sort_full(es, keys_np: np.ndarray, params=None, label=""):
    """Keys-only, pairs and argsort of one input against the oracle, element by element."""
    perm = oracle.stable_perm(keys_np)
    want = keys_np[perm]
    k = to_dev(keys_np)
    got = to_np(es.sort(k, params=params))
    assert_bits_equal(got, want, f"sort {label}")
    vals = (np.arange(keys_np.size, dtype=np.int64) * 2654435761 % (2**61)).astype(np.int64)
    k2, v2 = es.sort_pairs(k, to_dev(vals), params=params)
    assert_bits_equal(to_np(k2), want, f"sort_pairs keys {label}")
    assert_bits_equal(to_np(v2), vals[perm], f"sort_pairs values {label}")
    v32 = (np.arange(keys_np.size, dtype=np.int64) * 7 + 3).astype(np.int32)
    k3, v3 = es.sort_pairs(k, to_dev(v32), params=params)
    assert_bits_equal(to_np(k3), want, f"sort_pairs(4B) keys {label}")
    assert_bits_equal(to_np(v3), v32[perm], f"sort_pairs(4B) values {label}")
    torch = torch_mod()
    idx = to_np(es.argsort(k, params=params))
    assert np.array_equal(idx, perm), f"argsort int64 {label}"
    if keys_np.size < 2**31:
        idx32 = to_np(es.argsort(k, index_dtype=torch.int32, params=params))
        assert np.array_equal(idx32, perm.astype(np.int32)), f"argsort int32 {label}"
