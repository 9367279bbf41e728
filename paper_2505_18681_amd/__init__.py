"""EvoSort on AMD MI355X: Python binding of ``libevosort.so``.

This module only marshals arguments: it checks tensors, allocates the output
and scratch tensors with PyTorch on the keys' device, and calls the C ABI
declared in ``include/evosort.h`` on PyTorch's current stream.  Every step of
every sort runs in the library's HIP kernels; there is no CPU path.  Importing
the package fails if the library has not been built
(``python -m paper_2505_18681_amd.build``).

Public calls (names follow the C ABI):

* :func:`sort`, :func:`sort_pairs`, :func:`argsort` -- the three library sorts;
* :func:`radix_histogram`, :func:`radix_pass`, :func:`merge_block_sort`,
  :func:`merge_round` -- single steps of the two routines;
* :func:`segmented_sort`, :func:`segmented_sort_pairs` -- a batch of arrays
  (segments of one buffer) in one fixed launch sequence; :func:`sort_each`
  -- the same batch one plain sort per segment; :func:`segmented_stats`;
* :class:`Server` -- the request loop: admission by an HBM budget,
  continuous batching of short requests, overlapping jobs on several streams;
* :func:`plan`, :func:`temp_bytes`, :func:`default_params` -- host-only queries;
* :func:`profile_enable`, :func:`profile_reset`, :func:`profile_collect` --
  per-kernel HIP-event timing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libevosort.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_2505_18681_amd.build` first")

# PyTorch ships its own HIP runtime.  Load it first so that the library's
# dependency on libamdhip64.so.7 binds to that same runtime: two HIP runtimes
# in one process would not share devices, streams or allocations.
import torch  # noqa: E402,F401

_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants --
INT32, INT64, UINT32, FLOAT32, FLOAT64 = 1, 2, 3, 4, 5
ALGO_AUTO, ALGO_MERGE, ALGO_RADIX = 0, 3, 4
OP_SORT, OP_SORT_PAIRS, OP_ARGSORT = 0, 1, 2
PATH_NAMES = {0: "copy", 1: "small", 2: "radix", 3: "merge"}
(OK, ERR_INVALID_ARG, ERR_UNSUPPORTED_DTYPE, ERR_UNSUPPORTED_PARAM, ERR_TEMP_TOO_SMALL, ERR_HIP, ERR_DEVICE_TIMEOUT,
 ERR_OVER_BUDGET, ERR_PENDING) = range(9)
DEBUG_WITHHOLD_TILE0 = 0x1
DEBUG_WIDE_STATUS = 0x2

EXPORTED = (
    "evosort_default_params", "evosort_temp_bytes", "evosort_plan", "evosort_sort", "evosort_sort_pairs",
    "evosort_argsort", "evosort_radix_histogram", "evosort_radix_pass", "evosort_merge_block_sort",
    "evosort_merge_round", "evosort_status_string", "evosort_last_hip_error", "evosort_check_device_error",
    "evosort_profile_enable", "evosort_profile_reset", "evosort_profile_collect", "evosort_profile_get",
    "evosort_segmented_temp_bytes", "evosort_segmented_sort", "evosort_segmented_sort_pairs",
    "evosort_segmented_capacity", "evosort_segmented_stats", "evosort_sort_each",
    "evosort_server_default_config", "evosort_server_create", "evosort_server_destroy", "evosort_server_submit",
    "evosort_server_result", "evosort_server_wait", "evosort_server_copy_out", "evosort_server_times",
    "evosort_server_release", "evosort_server_drain", "evosort_server_get_stats", "evosort_build_id",
    "evosort_sort_noalloc", "evosort_stream_copy", "evosort_stream_read",
)


class Params(ctypes.Structure):
    """``evosort_params`` (see include/evosort.h)."""

    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("algo", ctypes.c_int32),
        ("digit_bits", ctypes.c_uint32),
        ("insertion_threshold", ctypes.c_uint32),
        ("fallback_threshold", ctypes.c_uint64),
        ("block_threads", ctypes.c_uint32),
        ("items_per_thread", ctypes.c_uint32),
        ("spin_limit", ctypes.c_uint32),
        ("debug_flags", ctypes.c_uint32),
        ("descending", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
    ]

    def __repr__(self):
        return "Params(" + ", ".join(f"{n}={getattr(self, n)}" for n, _ in self._fields_[1:-1]) + ")"


class PlanInfo(ctypes.Structure):
    """``evosort_plan_info`` (see include/evosort.h)."""

    _fields_ = [
        ("path", ctypes.c_int32),
        ("passes", ctypes.c_uint32),
        ("digit_bits", ctypes.c_uint32),
        ("block_threads", ctypes.c_uint32),
        ("items_per_thread", ctypes.c_uint32),
        ("status_bytes", ctypes.c_uint32),
        ("tile_keys", ctypes.c_uint64),
        ("tiles", ctypes.c_uint64),
        ("merge_rounds", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("merge_block_run", ctypes.c_uint64),
        ("small_capacity", ctypes.c_uint64),
        ("temp_bytes", ctypes.c_uint64),
    ]


class ServerConfig(ctypes.Structure):
    """``evosort_server_config`` (see include/evosort.h)."""

    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("streams", ctypes.c_uint32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("batch_max_keys", ctypes.c_uint64),
        ("batch_max_requests", ctypes.c_uint32),
        ("reserved", ctypes.c_uint32),
        ("params", Params),
    ]


class ServerStats(ctypes.Structure):
    """``evosort_server_stats`` (see include/evosort.h)."""

    _fields_ = [(name, ctypes.c_uint64) for name in (
        "submitted", "completed", "released", "failed", "jobs", "batched_requests", "keys_completed",
        "bytes_in_use", "peak_bytes", "budget_bytes")] + [
        ("max_concurrent_jobs", ctypes.c_uint32), ("waiting", ctypes.c_uint32)]


_vp, _i64, _u32, _i32, _sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
_P = ctypes.POINTER(Params)

_lib.evosort_default_params.argtypes = [_P]
_lib.evosort_default_params.restype = None
_lib.evosort_temp_bytes.argtypes = [_i32, _i32, _i64, _u32, _P, ctypes.POINTER(_sz)]
_lib.evosort_plan.argtypes = [_i32, _i32, _i64, _u32, _P, ctypes.POINTER(PlanInfo)]
_lib.evosort_sort.argtypes = [_i32, _vp, _vp, _i64, _vp, _sz, _P, _vp]
_lib.evosort_sort_pairs.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, _i64, _vp, _sz, _P, _vp]
_lib.evosort_argsort.argtypes = [_i32, _vp, _vp, _u32, _i64, _vp, _sz, _P, _vp]
_lib.evosort_sort_noalloc.argtypes = [_i32, _vp, _vp, _i64, _P, _vp]
_lib.evosort_sort_noalloc.restype = ctypes.c_int
_lib.evosort_stream_copy.argtypes = [_vp, _vp, _sz, _vp]
_lib.evosort_stream_copy.restype = ctypes.c_int
_lib.evosort_stream_read.argtypes = [_vp, _sz, _vp, _vp]
_lib.evosort_stream_read.restype = ctypes.c_int
_lib.evosort_radix_histogram.argtypes = [_i32, _vp, _i64, _u32, _vp, _vp, _vp, _sz, _vp]
_lib.evosort_radix_pass.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, _i64, _u32, _vp, _sz, _P, _vp]
_lib.evosort_merge_block_sort.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, _i64, _P, ctypes.POINTER(_i64), _vp]
_lib.evosort_merge_round.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, _i64, _i64, _vp, _sz, _vp]
_lib.evosort_status_string.argtypes = [_i32]
_lib.evosort_status_string.restype = ctypes.c_char_p
_lib.evosort_last_hip_error.argtypes = []
_lib.evosort_build_id.argtypes = []
_lib.evosort_build_id.restype = ctypes.c_char_p
_lib.evosort_check_device_error.argtypes = [_vp, _sz, _vp]
_lib.evosort_profile_enable.argtypes = [_i32]
_lib.evosort_profile_enable.restype = None
_lib.evosort_profile_reset.argtypes = []
_lib.evosort_profile_reset.restype = None
_lib.evosort_profile_collect.argtypes = []
_lib.evosort_profile_get.argtypes = [_i32, ctypes.c_char_p, _sz, ctypes.POINTER(ctypes.c_uint64),
                                     ctypes.POINTER(ctypes.c_double)]
_lib.evosort_segmented_temp_bytes.argtypes = [_i32, _i64, _i64, _u32, _P, ctypes.POINTER(_sz)]
_lib.evosort_segmented_sort.argtypes = [_i32, _vp, _vp, _i64, _vp, _i64, _vp, _sz, _P, _vp]
_lib.evosort_segmented_sort_pairs.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, _i64, _vp, _i64, _vp, _sz, _P, _vp]
_lib.evosort_segmented_capacity.argtypes = [_i32, _u32, ctypes.POINTER(_i64)]
_lib.evosort_segmented_stats.argtypes = [_vp, _sz, ctypes.POINTER(_u32), ctypes.POINTER(_u32), _vp]
_lib.evosort_sort_each.argtypes = [_i32, _vp, _vp, _vp, _vp, _u32, ctypes.POINTER(_i64), _i64, _vp, _sz, _P, _vp]
_SRV = ctypes.c_void_p
_lib.evosort_server_default_config.argtypes = [ctypes.POINTER(ServerConfig)]
_lib.evosort_server_default_config.restype = None
_lib.evosort_server_create.argtypes = [ctypes.POINTER(ServerConfig), ctypes.POINTER(_SRV)]
_lib.evosort_server_destroy.argtypes = [_SRV]
_lib.evosort_server_submit.argtypes = [_SRV, _i32, _vp, _i64, ctypes.POINTER(ctypes.c_uint64)]
_lib.evosort_server_result.argtypes = [_SRV, ctypes.c_uint64, ctypes.POINTER(_vp)]
_lib.evosort_server_wait.argtypes = [_SRV, ctypes.c_uint64, ctypes.POINTER(_vp)]
_lib.evosort_server_copy_out.argtypes = [_SRV, ctypes.c_uint64, _vp, _vp]
_lib.evosort_server_times.argtypes = [_SRV, ctypes.c_uint64] + [ctypes.POINTER(ctypes.c_double)] * 3
_lib.evosort_server_release.argtypes = [_SRV, ctypes.c_uint64]
_lib.evosort_server_drain.argtypes = [_SRV]
_lib.evosort_server_get_stats.argtypes = [_SRV, ctypes.POINTER(ServerStats)]
for _f in ("evosort_server_create", "evosort_server_destroy", "evosort_server_submit", "evosort_server_result",
           "evosort_server_wait", "evosort_server_copy_out", "evosort_server_times", "evosort_server_release",
           "evosort_server_drain", "evosort_server_get_stats"):
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("evosort_segmented_temp_bytes", "evosort_segmented_sort", "evosort_segmented_sort_pairs",
           "evosort_segmented_capacity", "evosort_segmented_stats", "evosort_sort_each"):
    getattr(_lib, _f).restype = ctypes.c_int
for _f in ("evosort_temp_bytes", "evosort_plan", "evosort_sort", "evosort_sort_pairs", "evosort_argsort",
           "evosort_radix_histogram", "evosort_radix_pass", "evosort_merge_block_sort", "evosort_merge_round",
           "evosort_last_hip_error", "evosort_check_device_error", "evosort_profile_collect", "evosort_profile_get"):
    getattr(_lib, _f).restype = ctypes.c_int


class EvosortError(RuntimeError):
    def __init__(self, where: str, status: int):
        self.status = status
        msg = status_string(status)
        if status == ERR_HIP:
            msg += f" (hipError_t {_lib.evosort_last_hip_error()})"
        super().__init__(f"{where}: {msg}")


def status_string(status: int) -> str:
    return _lib.evosort_status_string(int(status)).decode()


def build_id() -> str:
    """Hash of the sources the loaded library was compiled from (``evosort_build_id``)."""
    return _lib.evosort_build_id().decode()


def _check(where: str, st: int):
    if st != OK:
        raise EvosortError(where, st)


# ------------------------------------------------------------- host queries --
def default_params(**overrides) -> Params:
    """``evosort_default_params`` with keyword overrides (e.g. ``algo=ALGO_MERGE``)."""
    p = Params()
    _lib.evosort_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k) or k == "struct_size":
            raise AttributeError(f"no parameter {k!r}")
        setattr(p, k, v)
    return p


def _pp(params):
    return ctypes.byref(params) if params is not None else None


def temp_bytes(op: int, dtype_code: int, n: int, value_bytes: int = 0, params: Params | None = None) -> int:
    out = _sz(0)
    _check("evosort_temp_bytes", _lib.evosort_temp_bytes(op, dtype_code, n, value_bytes, _pp(params),
                                                         ctypes.byref(out)))
    return int(out.value)


def plan(op: int, dtype_code: int, n: int, value_bytes: int = 0, params: Params | None = None) -> dict:
    info = PlanInfo()
    _check("evosort_plan", _lib.evosort_plan(op, dtype_code, n, value_bytes, _pp(params), ctypes.byref(info)))
    d = {name: getattr(info, name) for name, _ in PlanInfo._fields_ if name != "reserved"}
    d["path_name"] = PATH_NAMES.get(info.path, "?")
    return d


# ------------------------------------------------------------ tensor helpers --
def _torch():
    import torch

    return torch


def dtype_code(dtype) -> int:
    torch = _torch()
    table = {torch.int32: INT32, torch.int64: INT64, torch.float32: FLOAT32, torch.float64: FLOAT64}
    if hasattr(torch, "uint32"):
        table[torch.uint32] = UINT32
    if dtype not in table:
        raise TypeError(f"evosort: unsupported key dtype {dtype}")
    return table[dtype]


def _key_tensor(t, what="keys"):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{what} must be on a GPU device (got {t.device}); the library has no CPU path")
    if t.dim() != 1 or not t.is_contiguous():
        raise ValueError(f"{what} must be a contiguous 1-D tensor")
    return t


def _stream(device, stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream(device)
    return ctypes.c_void_p(s.cuda_stream)


def _temp(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else None


def _finish(where: str, device, tmp, allocated, stream, check: bool):
    """After a call enqueued on ``stream``: tensors this module allocated on the current stream are marked
    as used by ``stream`` (so PyTorch's allocator does not hand their memory out again before that stream's
    kernels end), and with ``check`` the call's device error word is read (this synchronizes ``stream``)
    and a device-side failure raises."""
    torch = _torch()
    if stream is not None and stream.cuda_stream != torch.cuda.current_stream(device).cuda_stream:
        for t in (tmp, *allocated):
            if t is not None and t.numel():
                t.record_stream(stream)
    if check:
        with torch.cuda.device(device):
            _check(where, _lib.evosort_check_device_error(_ptr(tmp), tmp.numel(), _stream(device, stream)))


# ---------------------------------------------------------------- the sorts --
def sort(keys, *, params: Params | None = None, out=None, stream=None, temp=None, check: bool = False):
    """Keys in ascending order (stable; floats in IEEE totalOrder).  ``out=keys`` sorts in place.

    The call returns once the work is enqueued on ``stream`` (default: PyTorch's current stream).  With
    ``check=True`` it waits for the work and raises :class:`EvosortError` on a device-side failure; without,
    such a failure is raised by the next library call made after it happened."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    n = keys.numel()
    allocated = []
    if out is None:
        out = torch.empty_like(keys)
        allocated.append(out)
    _key_tensor(out, "out")
    if out.dtype != keys.dtype or out.numel() != n:
        raise ValueError("out must match keys in dtype and length")
    need = temp_bytes(OP_SORT, code, n, 0, params)
    tmp = temp if temp is not None else _temp(need, keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_sort", _lib.evosort_sort(code, _ptr(keys), _ptr(out), n, _ptr(tmp), tmp.numel(),
                                                 _pp(params), _stream(keys.device, stream)))
    _finish("evosort_sort", keys.device, tmp, allocated, stream, check)
    return out


def sort_pairs(keys, values, *, params: Params | None = None, keys_out=None, values_out=None, stream=None,
               temp=None, check: bool = False):
    """(keys, values) sorted stably by key; values are opaque 4- or 8-byte words.  ``stream`` and ``check``
    as for :func:`sort`."""
    torch = _torch()
    keys = _key_tensor(keys)
    values = _key_tensor(values, "values")
    code = dtype_code(keys.dtype)
    n = keys.numel()
    if values.numel() != n:
        raise ValueError("keys and values differ in length")
    vb = values.element_size()
    if vb not in (4, 8):
        raise TypeError("values must be 4- or 8-byte elements")
    allocated = []
    if keys_out is None:
        keys_out = torch.empty_like(keys)
        allocated.append(keys_out)
    if values_out is None:
        values_out = torch.empty_like(values)
        allocated.append(values_out)
    need = temp_bytes(OP_SORT_PAIRS, code, n, vb, params)
    tmp = temp if temp is not None else _temp(need, keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_sort_pairs",
               _lib.evosort_sort_pairs(code, _ptr(keys), _ptr(keys_out), _ptr(values), _ptr(values_out), vb, n,
                                       _ptr(tmp), tmp.numel(), _pp(params), _stream(keys.device, stream)))
    _finish("evosort_sort_pairs", keys.device, tmp, allocated, stream, check)
    return keys_out, values_out


def argsort(keys, *, index_dtype=None, params: Params | None = None, out=None, stream=None, temp=None,
            check: bool = False):
    """Stable sorting permutation (int64 by default, or int32).  ``stream`` and ``check`` as for :func:`sort`."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    n = keys.numel()
    index_dtype = index_dtype or torch.int64
    if index_dtype not in (torch.int32, torch.int64):
        raise TypeError("index_dtype must be torch.int32 or torch.int64")
    ib = 4 if index_dtype == torch.int32 else 8
    allocated = []
    if out is None:
        out = torch.empty(n, dtype=index_dtype, device=keys.device)
        allocated.append(out)
    need = temp_bytes(OP_ARGSORT, code, n, ib, params)
    tmp = temp if temp is not None else _temp(need, keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_argsort", _lib.evosort_argsort(code, _ptr(keys), _ptr(out), ib, n, _ptr(tmp), tmp.numel(),
                                                       _pp(params), _stream(keys.device, stream)))
    _finish("evosort_argsort", keys.device, tmp, allocated, stream, check)
    return out


NOALLOC_SCRATCH_BYTES = 64 << 20  # EVOSORT_NOALLOC_SCRATCH_BYTES


def sort_noalloc(keys, *, params: Params | None = None, out=None, stream=None):
    """:func:`sort` through ``evosort_sort_noalloc``: the library takes no scratch from the caller and allocates
    nothing (its scratch is a device array of ``NOALLOC_SCRATCH_BYTES`` inside the library, shared by every
    such call on the device, so calls that overlap in time on one device race).  Only ``out``, when not
    given, is allocated here."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    allocated = []
    if out is None:
        out = torch.empty_like(keys)
        allocated.append(out)
    _key_tensor(out, "out")
    if out.dtype != keys.dtype or out.numel() != keys.numel():
        raise ValueError("out must match keys in dtype and length")
    with torch.cuda.device(keys.device):
        _check("evosort_sort_noalloc", _lib.evosort_sort_noalloc(code, _ptr(keys), _ptr(out), keys.numel(),
                                                                 _pp(params), _stream(keys.device, stream)))
    _finish("evosort_sort_noalloc", keys.device, None, allocated, stream, False)
    return out


# ------------------------------------------------------------ single steps --
def radix_histogram(keys, digit_bits: int = 8, *, stream=None):
    """(hist, bases): uint64-valued int64 tensors of shape (passes, 2**digit_bits)."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    passes = (8 * keys.element_size() + digit_bits - 1) // digit_bits
    hist = torch.empty((passes, 1 << digit_bits), dtype=torch.int64, device=keys.device)
    bases = torch.empty_like(hist)
    with torch.cuda.device(keys.device):
        _check("evosort_radix_histogram",
               _lib.evosort_radix_histogram(code, _ptr(keys), keys.numel(), digit_bits, _ptr(hist), _ptr(bases),
                                            None, 0, _stream(keys.device, stream)))
    _finish("evosort_radix_histogram", keys.device, None, [hist, bases], stream, False)
    return hist, bases


def radix_pass(keys, values=None, *, pass_index: int, params: Params | None = None, stream=None):
    """One stable LSD pass on digit ``pass_index``: returns (keys_out, values_out or None)."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    n = keys.numel()
    vb = 0 if values is None else _key_tensor(values, "values").element_size()
    op = OP_SORT_PAIRS if vb else OP_SORT
    kout = torch.empty_like(keys)
    vout = torch.empty_like(values) if vb else None
    tmp = _temp(temp_bytes(op, code, n, vb, params), keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_radix_pass",
               _lib.evosort_radix_pass(code, _ptr(keys), _ptr(kout), _ptr(values) if vb else None,
                                       _ptr(vout) if vb else None, vb, n, pass_index, _ptr(tmp), tmp.numel(),
                                       _pp(params), _stream(keys.device, stream)))
    _finish("evosort_radix_pass", keys.device, tmp, [kout, vout], stream, False)
    return kout, vout


def merge_block_sort(keys, values=None, *, params: Params | None = None, stream=None):
    """Mergesort block sort: returns (keys_out, values_out or None, run_length)."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    n = keys.numel()
    vb = 0 if values is None else _key_tensor(values, "values").element_size()
    kout = torch.empty_like(keys)
    vout = torch.empty_like(values) if vb else None
    run = _i64(0)
    with torch.cuda.device(keys.device):
        _check("evosort_merge_block_sort",
               _lib.evosort_merge_block_sort(code, _ptr(keys), _ptr(kout), _ptr(values) if vb else None,
                                             _ptr(vout) if vb else None, vb, n, _pp(params), ctypes.byref(run),
                                             _stream(keys.device, stream)))
    _finish("evosort_merge_block_sort", keys.device, None, [kout, vout], stream, False)
    return kout, vout, int(run.value)


def merge_round(keys, values=None, *, run: int, stream=None):
    """One merge round over pairs of sorted runs of length ``run``: returns (keys_out, values_out or None)."""
    torch = _torch()
    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    n = keys.numel()
    vb = 0 if values is None else _key_tensor(values, "values").element_size()
    op = OP_SORT_PAIRS if vb else OP_SORT
    kout = torch.empty_like(keys)
    vout = torch.empty_like(values) if vb else None
    tmp = _temp(256 + 8 * (n + 4), keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_merge_round",
               _lib.evosort_merge_round(code, _ptr(keys), _ptr(kout), _ptr(values) if vb else None,
                                        _ptr(vout) if vb else None, vb, n, run, _ptr(tmp), tmp.numel(),
                                        _stream(keys.device, stream)))
    _finish("evosort_merge_round", keys.device, tmp, [kout, vout], stream, False)
    return kout, vout


# ---------------------------------------------------------- batches of arrays --
def segmented_temp_bytes(dtype_code_: int, n: int, nseg: int, value_bytes: int = 0,
                         params: Params | None = None) -> int:
    out = _sz(0)
    _check("evosort_segmented_temp_bytes",
           _lib.evosort_segmented_temp_bytes(dtype_code_, n, nseg, value_bytes, _pp(params), ctypes.byref(out)))
    return int(out.value)


def segmented_capacity(dtype_code_: int, value_bytes: int = 0) -> int:
    """Largest segment the one-workgroup classes sort."""
    out = _i64(0)
    _check("evosort_segmented_capacity", _lib.evosort_segmented_capacity(dtype_code_, value_bytes,
                                                                         ctypes.byref(out)))
    return int(out.value)


def _offsets_tensor(offsets, device):
    torch = _torch()
    if not isinstance(offsets, torch.Tensor):
        raise TypeError("offsets must be a torch.Tensor of int64 on the keys' device")
    if offsets.dtype != torch.int64 or offsets.dim() != 1 or not offsets.is_contiguous():
        raise ValueError("offsets must be a contiguous 1-D int64 tensor")
    if offsets.device != device:
        raise ValueError(f"offsets must be on {device} (got {offsets.device})")
    if offsets.numel() < 1:
        raise ValueError("offsets needs nseg + 1 >= 1 entries")
    return offsets


def segmented_sort(keys, offsets, *, params: Params | None = None, out=None, stream=None, temp=None,
                   check: bool = False):
    """Each segment keys[offsets[i]:offsets[i+1]] sorted on its own (stable), in one launch sequence.

    ``offsets`` is an int64 tensor on the keys' device.  Positions outside
    [offsets[0], offsets[-1]) of ``out`` are left as they are.
    """
    torch = _torch()
    keys = _key_tensor(keys)
    offsets = _offsets_tensor(offsets, keys.device)
    code = dtype_code(keys.dtype)
    n, nseg = keys.numel(), offsets.numel() - 1
    allocated = []
    if out is None:
        out = torch.empty_like(keys)
        allocated.append(out)
    _key_tensor(out, "out")
    if out.dtype != keys.dtype or out.numel() != n:
        raise ValueError("out must match keys in dtype and length")
    tmp = temp if temp is not None else _temp(segmented_temp_bytes(code, n, nseg, 0, params), keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_segmented_sort",
               _lib.evosort_segmented_sort(code, _ptr(keys), _ptr(out), n, _ptr(offsets), nseg, _ptr(tmp),
                                           tmp.numel(), _pp(params), _stream(keys.device, stream)))
    _finish("evosort_segmented_sort", keys.device, tmp, allocated, stream, check)
    return out


def segmented_sort_pairs(keys, values, offsets, *, params: Params | None = None, keys_out=None, values_out=None,
                         stream=None, temp=None, check: bool = False):
    """(keys, values) with each segment sorted stably by key, in one launch sequence."""
    torch = _torch()
    keys = _key_tensor(keys)
    values = _key_tensor(values, "values")
    offsets = _offsets_tensor(offsets, keys.device)
    code = dtype_code(keys.dtype)
    n, nseg = keys.numel(), offsets.numel() - 1
    if values.numel() != n:
        raise ValueError("keys and values differ in length")
    vb = values.element_size()
    if vb not in (4, 8):
        raise TypeError("values must be 4- or 8-byte elements")
    allocated = []
    if keys_out is None:
        keys_out = torch.empty_like(keys)
        allocated.append(keys_out)
    if values_out is None:
        values_out = torch.empty_like(values)
        allocated.append(values_out)
    tmp = temp if temp is not None else _temp(segmented_temp_bytes(code, n, nseg, vb, params), keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_segmented_sort_pairs",
               _lib.evosort_segmented_sort_pairs(code, _ptr(keys), _ptr(keys_out), _ptr(values), _ptr(values_out),
                                                 vb, n, _ptr(offsets), nseg, _ptr(tmp), tmp.numel(), _pp(params),
                                                 _stream(keys.device, stream)))
    _finish("evosort_segmented_sort_pairs", keys.device, tmp, allocated, stream, check)
    return keys_out, values_out


def segmented_stats(temp, *, stream=None) -> dict:
    """What the last segmented call on ``temp`` did (synchronizes): class counts and radix tiles."""
    torch = _torch()
    counts = (_u32 * 5)()
    tiles = _u32(0)
    with torch.cuda.device(temp.device):
        _check("evosort_segmented_stats", _lib.evosort_segmented_stats(_ptr(temp), temp.numel(), counts,
                                                                       ctypes.byref(tiles),
                                                                       _stream(temp.device, stream)))
    return {"block_classes": [int(c) for c in counts[:4]], "large": int(counts[4]), "tiles": int(tiles.value)}


def sort_each(keys, host_offsets, values=None, *, params: Params | None = None, out=None, values_out=None,
              stream=None, temp=None):
    """The batch sorted one plain sort per segment (``host_offsets``: a host sequence of nseg + 1 ints)."""
    torch = _torch()
    import numpy as np

    keys = _key_tensor(keys)
    code = dtype_code(keys.dtype)
    offs = np.ascontiguousarray(np.asarray(host_offsets, dtype=np.int64))
    nseg = offs.size - 1
    allocated = []
    if out is None:
        out = torch.empty_like(keys)
        allocated.append(out)
    vb = 0
    if values is not None:
        values = _key_tensor(values, "values")
        vb = values.element_size()
        if values_out is None:
            values_out = torch.empty_like(values)
            allocated.append(values_out)
    longest = int(np.max(np.diff(offs))) if nseg > 0 else 0
    op = OP_SORT_PAIRS if vb else OP_SORT
    tmp = temp if temp is not None else _temp(temp_bytes(op, code, longest, vb, params), keys.device)
    with torch.cuda.device(keys.device):
        _check("evosort_sort_each",
               _lib.evosort_sort_each(code, _ptr(keys), _ptr(out), _ptr(values) if vb else None,
                                      _ptr(values_out) if vb else None, vb,
                                      offs.ctypes.data_as(ctypes.POINTER(_i64)), nseg, _ptr(tmp), tmp.numel(),
                                      _pp(params), _stream(keys.device, stream)))
    _finish("evosort_sort_each", keys.device, tmp, allocated, stream, False)
    return (out, values_out) if vb else out


def check_device_error(temp, *, stream=None) -> int:
    """Synchronize and read the error word a radix call left in ``temp``: a status code."""
    torch = _torch()
    with torch.cuda.device(temp.device):
        return _lib.evosort_check_device_error(_ptr(temp), temp.numel(), _stream(temp.device, stream))


# ------------------------------------------------------------------ serving --
def server_default_config(**overrides) -> ServerConfig:
    """``evosort_server_default_config`` with keyword overrides (``params`` takes a :class:`Params`)."""
    c = ServerConfig()
    _lib.evosort_server_default_config(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise AttributeError(f"evosort_server_config has no field {k!r}")
        setattr(c, k, v)
    return c


class Server:
    """A sort server on the current device (``evosort_server_*``).

    ``submit`` takes a device tensor of keys (kept alive by the server object
    until the request is released) and returns a request id; ``wait`` /
    ``done`` report completion; ``result`` copies the sorted keys into a new
    tensor on PyTorch's current stream; ``release`` frees the request's HBM.
    """

    def __init__(self, *, hbm_budget_bytes: int = 1 << 30, streams: int = 4, batch_max_keys: int = 65536,
                 batch_max_requests: int = 2048, params: Params | None = None, device=None):
        torch = _torch()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        cfg = server_default_config(hbm_budget_bytes=int(hbm_budget_bytes), streams=int(streams),
                                    batch_max_keys=int(batch_max_keys), batch_max_requests=int(batch_max_requests))
        if params is not None:
            cfg.params = params
        self._h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check("evosort_server_create", _lib.evosort_server_create(ctypes.byref(cfg), ctypes.byref(self._h)))
        self._inputs = {}

    def close(self):
        if self._h:
            _check("evosort_server_destroy", _lib.evosort_server_destroy(self._h))
            self._h = ctypes.c_void_p()
            self._inputs.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def submit(self, keys) -> int:
        keys = _key_tensor(keys)
        if keys.device != self.device:
            raise ValueError(f"keys must be on {self.device}")
        rid = ctypes.c_uint64(0)
        # the keys must be in HBM before the server's streams read them
        _torch().cuda.current_stream(self.device).synchronize()
        _check("evosort_server_submit", _lib.evosort_server_submit(self._h, dtype_code(keys.dtype), _ptr(keys),
                                                                   keys.numel(), ctypes.byref(rid)))
        self._inputs[rid.value] = keys
        return rid.value

    def done(self, rid: int) -> bool:
        st = _lib.evosort_server_result(self._h, rid, None)
        if st == ERR_PENDING:
            return False
        _check("evosort_server_result", st)
        return True

    def wait(self, rid: int):
        _check("evosort_server_wait", _lib.evosort_server_wait(self._h, rid, None))

    def result(self, rid: int, out=None):
        """The sorted keys of a finished request, copied into ``out`` (or a new tensor)."""
        torch = _torch()
        keys = self._inputs[rid]
        out = torch.empty_like(keys) if out is None else out
        if out.numel() != keys.numel() or out.dtype != keys.dtype:
            raise ValueError("out must match the request's keys")
        self.wait(rid)
        _check("evosort_server_copy_out",
               _lib.evosort_server_copy_out(self._h, rid, _ptr(out), _stream(self.device, None)))
        return out

    def times(self, rid: int) -> tuple:
        """(submitted, admitted, finished) in ms since the server was created."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check("evosort_server_times", _lib.evosort_server_times(self._h, rid, ctypes.byref(a), ctypes.byref(b),
                                                                 ctypes.byref(c)))
        return a.value, b.value, c.value

    def release(self, rid: int):
        _check("evosort_server_release", _lib.evosort_server_release(self._h, rid))
        self._inputs.pop(rid, None)

    def drain(self):
        _check("evosort_server_drain", _lib.evosort_server_drain(self._h))

    def stats(self) -> dict:
        s = ServerStats()
        _check("evosort_server_get_stats", _lib.evosort_server_get_stats(self._h, ctypes.byref(s)))
        return {name: int(getattr(s, name)) for name, _ in ServerStats._fields_}


# -------------------------------------------------------- streaming ceilings --
def stream_copy(dst, src, *, stream=None):
    """``evosort_stream_copy``: copy tensor ``src`` into ``dst`` (same number of bytes) with the library's
    streaming copy kernel (reads and writes every byte once)."""
    torch = _torch()
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst and src must be contiguous and of the same size in bytes")
    with torch.cuda.device(src.device):
        _check("evosort_stream_copy", _lib.evosort_stream_copy(_ptr(dst), _ptr(src), nbytes,
                                                               _stream(src.device, stream)))
    return dst


def stream_read(src, sink, *, stream=None):
    """``evosort_stream_read``: read every byte of ``src`` once (``sink``: an 8-byte device tensor)."""
    torch = _torch()
    with torch.cuda.device(src.device):
        _check("evosort_stream_read", _lib.evosort_stream_read(_ptr(src), src.numel() * src.element_size(),
                                                               _ptr(sink), _stream(src.device, stream)))


# --------------------------------------------------------------- profiling --
def profile_enable(on: bool = True):
    _lib.evosort_profile_enable(1 if on else 0)


def profile_reset():
    _lib.evosort_profile_reset()


def profile_collect() -> dict:
    """{kernel name: (launches, total milliseconds)} for every launch since the last reset."""
    count = _lib.evosort_profile_collect()
    out = {}
    name = ctypes.create_string_buffer(128)
    for i in range(count):
        launches = ctypes.c_uint64(0)
        ms = ctypes.c_double(0.0)
        _check("evosort_profile_get", _lib.evosort_profile_get(i, name, 128, ctypes.byref(launches),
                                                               ctypes.byref(ms)))
        out[name.value.decode()] = (int(launches.value), float(ms.value))
    return out
