"""Host-side checks of the C ABI (no GPU needed).

* the library loads and exports every function include/evosort.h declares;
* the dispatch of the adaptive partition sort (Sec. 4.3, Algorithm 6) in
  evosort_plan agrees with the oracle's rule and the paper's branch table;
* plan shapes (passes per digit width, look-back word width, merge rounds);
* argument errors are returned synchronously, before anything touches a GPU.
"""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
from conftest import ROOT, read_golden

es = pytest.importorskip("paper_2505_18681_amd")

HEADER = os.path.join(ROOT, "include", "evosort.h")
DTYPES = {"int32": es.INT32, "int64": es.INT64, "uint32": es.UINT32, "float32": es.FLOAT32, "float64": es.FLOAT64}


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(evosort_[a-z0-9_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported():
    names = declared_functions()
    assert len(names) >= 17
    out = subprocess.run(["nm", "-D", "--defined-only", es.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s+(evosort_\w+)", out))
    assert set(names) <= exported, set(names) - exported
    assert exported <= set(names), f"exported but undeclared: {exported - set(names)}"
    assert set(es.EXPORTED) == set(names)
    lib = ctypes.CDLL(es.LIB_PATH)
    for nm in names:
        assert hasattr(lib, nm)


def test_loaded_library_is_built_from_this_tree():
    """The library reports the hash of the sources it was compiled from; it must be the tree's current one."""
    import importlib.util

    spec = importlib.util.spec_from_file_location("_evosort_build_script",
                                                  os.path.join(ROOT, "paper_2505_18681_amd", "build.py"))
    build = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(build)
    assert re.fullmatch(r"[0-9a-f]{16}", es.build_id())
    assert es.build_id() == build.source_hash(), "libevosort.so is stale: rebuild it"


def test_only_abi_symbols_are_exported():
    out = subprocess.run(["nm", "-D", "--defined-only", es.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    funcs = re.findall(r"\sT\s+(\S+)", out)
    assert all(f.startswith("evosort_") for f in funcs), [f for f in funcs if not f.startswith("evosort_")]


def test_default_params():
    p = es.default_params()
    assert p.struct_size == ctypes.sizeof(es.Params)
    assert p.algo == es.ALGO_AUTO and p.digit_bits == 8
    assert 1 <= p.insertion_threshold <= 2048
    assert p.fallback_threshold >= 1


def test_status_strings():
    for st in range(7):
        assert es.status_string(st)
    assert es.status_string(0) == "ok"
    assert "unknown" in es.status_string(99)


def test_dispatch_matches_oracle_rule():
    """Algorithm 6 as the oracle states it, with A_code 0 read as the compiled GA table's routine for the key
    type and length (the mergesort where a row picked it, radix elsewhere)."""
    from paper_2505_18681_amd import tuner

    merge_rows = [r for r in tuner.auto_table_rows(tuner.packaged_table()) if r[4] == es.ALGO_MERGE]
    for dt_name, code in DTYPES.items():
        integer = dt_name != "float32" and dt_name != "float64"
        for algo in (es.ALGO_AUTO, es.ALGO_MERGE, es.ALGO_RADIX):
            for fb in (0, 1, 2, 100, 5000, 16384, 10**6):
                p = es.default_params(algo=algo, fallback_threshold=fb)
                for n in (0, 1, 2, 3, 99, 100, 101, 4999, 5000, 8191, 8192, 8193, 16383, 16384, 50_000, 10**6):
                    info = es.plan(es.OP_SORT, code, n, 0, p)
                    if n <= 1:
                        assert info["path_name"] == "copy"
                        continue
                    a = algo
                    if algo == es.ALGO_AUTO and any(r[0] == dt_name and r[2] <= n < r[3] for r in merge_rows):
                        a = es.ALGO_MERGE
                    want = oracle.aps_path(n, integer, a, fb, info["small_capacity"], radix_for_floats=True)
                    assert info["path_name"] == want, (dt_name, algo, fb, n)


def test_dispatch_follows_the_papers_branch_table(golden):
    """Alg. 6 rows for integer keys (the paper's radix branch is for integers)."""
    for n, t_np, a_code, is_int, expect in golden("aps_dispatch.txt"):
        n, t_np, a_code, is_int = int(n), int(t_np), int(a_code), int(is_int)
        if not is_int or a_code not in (3, 4) or n <= 1:
            continue  # float keys and other codes are readings of the library (tested above / below)
        p = es.default_params(algo=a_code, fallback_threshold=t_np)
        info = es.plan(es.OP_SORT, es.INT32, n, 0, p)
        if n >= info["small_capacity"] and expect == "small":
            continue  # the one-workgroup sort caps the small branch (a reading of the library)
        assert info["path_name"] == expect, (n, t_np, a_code)


def test_unknown_algo_codes_are_rejected():
    for code in (1, 2, 5, 7, -1):
        with pytest.raises(es.EvosortError) as e:
            es.plan(es.OP_SORT, es.INT32, 1000, 0, es.default_params(algo=code))
        assert e.value.status == es.ERR_INVALID_ARG


@pytest.mark.parametrize("bits", range(4, 13))
def test_pass_counts(bits):
    p = es.default_params(digit_bits=bits, fallback_threshold=0)
    for code, kb in ((es.INT32, 4), (es.INT64, 8)):
        info = es.plan(es.OP_SORT, code, 10**6, 0, p)
        assert info["passes"] == -(-8 * kb // bits)
        assert info["passes"] == oracle.pass_count(np.int32 if kb == 4 else np.int64, bits)


def test_status_word_width_switch():
    p = es.default_params(fallback_threshold=0)
    assert es.plan(es.OP_SORT, es.INT32, (1 << 30) - 1, 0, p)["status_bytes"] == 4
    assert es.plan(es.OP_SORT, es.INT32, 1 << 30, 0, p)["status_bytes"] == 8
    assert es.plan(es.OP_SORT, es.INT32, 10**10, 0, p)["status_bytes"] == 8


def test_merge_plan_schedule():
    for t_ins in (1, 2, 3, 17, 195, 629, 2048):
        p = es.default_params(algo=es.ALGO_MERGE, fallback_threshold=0, insertion_threshold=t_ins)
        for n in (2, 4096, 10**6, 10**8):
            info = es.plan(es.OP_SORT, es.INT32, n, 0, p)
            run = info["merge_block_run"]
            assert run % t_ins == 0
            m = run // t_ins
            assert m & (m - 1) == 0 and run <= 4096 and 2 * run > 4096
            rounds = 0
            while run < n:
                run *= 2
                rounds += 1
            assert info["merge_rounds"] == rounds


def test_temp_bytes_cover_both_routines():
    for op, vb in ((es.OP_SORT, 0), (es.OP_SORT_PAIRS, 4), (es.OP_SORT_PAIRS, 8), (es.OP_ARGSORT, 4)):
        for n in (2, 10**4, 10**6):
            t = es.temp_bytes(op, es.INT64, n, vb)
            for algo in (es.ALGO_RADIX, es.ALGO_MERGE):
                p = es.default_params(algo=algo, fallback_threshold=0)
                assert es.plan(op, es.INT64, n, vb, p)["temp_bytes"] <= max(t, es.temp_bytes(op, es.INT64, n, vb, p))


# ---------------------------------------------------------- argument errors --
FAKE = 0x7F0000000000  # never dereferenced: every call below fails validation first


def _sort(code, kin, kout, n, temp, tb, params=None):
    return es._lib.evosort_sort(code, kin, kout, n, temp, tb, ctypes.byref(params) if params else None, None)


def test_argument_errors_are_synchronous():
    big = 1 << 40
    assert _sort(es.INT32, FAKE, FAKE + big, -1, FAKE + 2 * big, big) == es.ERR_INVALID_ARG
    assert _sort(99, FAKE, FAKE + big, 10, FAKE + 2 * big, big) == es.ERR_UNSUPPORTED_DTYPE
    assert _sort(es.INT32, None, FAKE + big, 10**6, FAKE + 2 * big, big) == es.ERR_INVALID_ARG
    assert _sort(es.INT32, FAKE, None, 10**6, FAKE + 2 * big, big) == es.ERR_INVALID_ARG
    need = es.temp_bytes(es.OP_SORT, es.INT32, 10**6)
    assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + 2 * big, need - 1) == es.ERR_TEMP_TOO_SMALL
    # misaligned temp
    assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + 2 * big + 8, need) == es.ERR_INVALID_ARG
    # output overlapping the input without being the same buffer
    assert _sort(es.INT32, FAKE, FAKE + 4, 10**6, FAKE + 2 * big, need) == es.ERR_INVALID_ARG
    # temp overlapping the output
    assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + big + 256, need) == es.ERR_INVALID_ARG
    # bad parameters
    for kw in ({"digit_bits": 3}, {"digit_bits": 13}, {"insertion_threshold": 0}, {"insertion_threshold": 4096},
               {"block_threads": 256}, {"algo": 2}):
        p = es.default_params(**kw)
        assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + 2 * big, big, p) == es.ERR_INVALID_ARG, kw
    bad = es.default_params()
    bad.struct_size = 4
    assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + 2 * big, big, bad) == es.ERR_INVALID_ARG
    # a tile shape that is not compiled in
    p = es.default_params(block_threads=128, items_per_thread=7, fallback_threshold=0)
    assert _sort(es.INT32, FAKE, FAKE + big, 10**6, FAKE + 2 * big, big, p) == es.ERR_UNSUPPORTED_PARAM
    # n = 0 is a no-op even with null pointers
    assert _sort(es.INT32, None, None, 0, None, 0) == es.OK


def test_pairs_and_argsort_argument_errors():
    big = 1 << 40
    lib = es._lib
    # value width
    assert lib.evosort_sort_pairs(es.INT32, FAKE, FAKE + big, FAKE + 2 * big, FAKE + 3 * big, 2, 100,
                                  FAKE + 4 * big, big, None, None) == es.ERR_UNSUPPORTED_DTYPE
    # values aliasing keys
    assert lib.evosort_sort_pairs(es.INT32, FAKE, FAKE + big, FAKE, FAKE + 3 * big, 4, 10**6,
                                  FAKE + 4 * big, big, None, None) == es.ERR_INVALID_ARG
    # int32 indices for more than 2^31 - 1 keys
    assert lib.evosort_argsort(es.INT32, FAKE, FAKE + big, 4, 2**31, FAKE + 2 * big, 1 << 45, None,
                               None) == es.ERR_INVALID_ARG
    assert lib.evosort_argsort(es.INT32, FAKE, FAKE + big, 3, 100, FAKE + 2 * big, big, None,
                               None) == es.ERR_UNSUPPORTED_DTYPE
    # steps
    assert lib.evosort_radix_pass(es.INT32, FAKE, FAKE + big, None, None, 0, 1000, 4, FAKE + 2 * big, big, None,
                                  None) == es.ERR_INVALID_ARG  # pass index out of range
    assert lib.evosort_merge_round(es.INT32, FAKE, FAKE + big, None, None, 0, 1000, 0, FAKE + 2 * big, big,
                                   None) == es.ERR_INVALID_ARG  # run < 1
    assert lib.evosort_radix_histogram(es.INT32, FAKE, 1000, 3, FAKE + big, None, None, 0,
                                       None) == es.ERR_INVALID_ARG


def test_segmented_plan_and_argument_errors():
    big = 1 << 40
    lib = es._lib
    assert es.segmented_capacity(es.UINT32, 0) == 16384
    assert es.segmented_capacity(es.INT64, 0) == es.segmented_capacity(es.INT32, 4) == 8192
    assert es.segmented_capacity(es.FLOAT64, 8) == es.segmented_capacity(es.FLOAT32, 8) == 4096
    # scratch grows with n and with the number of segments
    t1 = es.segmented_temp_bytes(es.UINT32, 10**6, 100)
    assert es.segmented_temp_bytes(es.UINT32, 2 * 10**6, 100) > t1
    assert es.segmented_temp_bytes(es.UINT32, 10**6, 1000) > t1
    assert es.segmented_temp_bytes(es.UINT32, 10**6, 100, 4) > t1
    # the segmented routine is radix-only with 8-bit digits
    for kw in ({"digit_bits": 11}, {"algo": es.ALGO_MERGE}, {"block_threads": 128, "items_per_thread": 7}):
        with pytest.raises(es.EvosortError) as e:
            es.segmented_temp_bytes(es.UINT32, 10**6, 100, 0, es.default_params(**kw))
        assert e.value.status == es.ERR_UNSUPPORTED_PARAM, kw
    need = es.segmented_temp_bytes(es.UINT32, 10**6, 100)
    seg = lib.evosort_segmented_sort
    assert seg(es.UINT32, FAKE, FAKE + big, 10**6, FAKE + 3 * big, -1, FAKE + 2 * big, need, None,
               None) == es.ERR_INVALID_ARG
    assert seg(es.UINT32, FAKE, FAKE + big, 10**6, None, 100, FAKE + 2 * big, need, None, None) == es.ERR_INVALID_ARG
    assert seg(es.UINT32, FAKE, FAKE + big, 10**6, FAKE + 3 * big, 100, FAKE + 2 * big, need - 1, None,
               None) == es.ERR_TEMP_TOO_SMALL
    assert seg(99, FAKE, FAKE + big, 10**6, FAKE + 3 * big, 100, FAKE + 2 * big, need, None,
               None) == es.ERR_UNSUPPORTED_DTYPE
    # offsets inside the keys, temp overlapping the output
    assert seg(es.UINT32, FAKE, FAKE + big, 10**6, FAKE + 64, 100, FAKE + 2 * big, need, None,
               None) == es.ERR_INVALID_ARG
    assert seg(es.UINT32, FAKE, FAKE + big, 10**6, FAKE + 3 * big, 100, FAKE + big + 256, need, None,
               None) == es.ERR_INVALID_ARG
    assert lib.evosort_segmented_sort_pairs(es.UINT32, FAKE, FAKE + big, FAKE + 4 * big, FAKE + 5 * big, 2, 10**6,
                                            FAKE + 3 * big, 100, FAKE + 2 * big, big, None,
                                            None) == es.ERR_UNSUPPORTED_DTYPE
    # one-by-one schedule: host offsets are checked before anything is enqueued
    offs = (ctypes.c_int64 * 3)(0, 10, 5)
    assert lib.evosort_sort_each(es.UINT32, FAKE, FAKE + big, None, None, 0, offs, 2, FAKE + 2 * big, big, None,
                                 None) == es.ERR_INVALID_ARG


def test_server_config_defaults_and_validation():
    """The server's config checks run on the host before any device call."""
    import ctypes

    import paper_2505_18681_amd as es

    c = es.server_default_config()
    assert c.struct_size == ctypes.sizeof(es.ServerConfig)
    assert (c.streams, c.hbm_budget_bytes, c.batch_max_keys, c.batch_max_requests) == (4, 1 << 30, 65536, 2048)
    assert c.params.digit_bits == 8
    h = ctypes.c_void_p()
    for bad in (dict(streams=0), dict(streams=17), dict(batch_max_requests=0), dict(batch_max_requests=9000),
                dict(hbm_budget_bytes=4096), dict(batch_max_keys=1 << 30)):
        cfg = es.server_default_config(**bad)
        assert es._lib.evosort_server_create(ctypes.byref(cfg), ctypes.byref(h)) == es.ERR_INVALID_ARG, bad
    cfg = es.server_default_config()
    cfg.struct_size = 8
    assert es._lib.evosort_server_create(ctypes.byref(cfg), ctypes.byref(h)) == es.ERR_INVALID_ARG
    assert es._lib.evosort_server_submit(None, es.INT32, None, 0, None) == es.ERR_INVALID_ARG
    assert es.status_string(es.ERR_OVER_BUDGET).startswith("request")
    assert es.status_string(es.ERR_PENDING).startswith("request")


@pytest.mark.parametrize("n, shape, pair_shape", [
    (2_097_152, (768, 12), (768, 12)),      # 2^21: the mid-size tile of every width
    (2_097_153, (768, 16), (768, 16)),      # 171 tiles of 12288 keys: every tile on its own CU
    (2_462_681, (768, 16), (768, 16)),
    (3_427_305, (768, 20), (768, 20)),      # 224 tiles of 15360
    (4_043_198, (1024, 16), (1024, 16)),    # 247 tiles of 16384
    (4_769_769, (1024, 20), (768, 16)),     # 233 tiles of 20480 (not compiled with values: 389 of 12288)
    (5_626_906, (768, 16), (768, 16)),      # 458 tiles: 2 per CU, 24576 keys on the busiest
    (8_388_608, (1024, 16), (1024, 16)),    # 2^23: 512 tiles, 2 per CU
    (8_388_609, (768, 24), (768, 24)),      # above 2^23 only 768 x 24 and 1024 x 16 compete: 456 tiles against 513
    (10_000_000, (1024, 16), (1024, 16)),   # 611 tiles, 3 per CU: 49152 keys on the busiest against 55296
    (12_647_247, (768, 24), (768, 24)),     # 687 tiles against 772
    (67_108_864, (1024, 16), (1024, 16)),   # 2^26: 4096 tiles, 16 per CU
    (67_108_865, (768, 24), (768, 24)),     # above 2^26: the large-array tile
])
def test_default_tile_follows_the_cu_count(n, shape, pair_shape):
    """4-byte keys between 2^21 and 2^26 keys, alone or with 4-byte values (or 32-bit argsort indices), take the
    tile that puts the fewest keys on the busiest of the 256 CUs among the shapes compiled for them
    (hand-computed); pairs with an 8-byte word take fixed mid-size tiles there, 8-byte keys alone keep theirs."""
    p = es.default_params(algo=es.ALGO_RADIX)

    def tile(op, code, vb):
        info = es.plan(op, code, n, vb, p)
        return info["block_threads"], info["items_per_thread"]

    assert tile(es.OP_SORT, es.INT32, 0) == shape
    assert tile(es.OP_SORT, es.FLOAT32, 0) == shape
    assert tile(es.OP_SORT_PAIRS, es.INT32, 4) == pair_shape
    assert tile(es.OP_ARGSORT, es.UINT32, 4) == pair_shape
    # an 8-byte word among key and value: fixed mid-size tiles between 2^21 and 2^26 keys
    mid = 1 << 21 < n <= 1 << 26
    small = n <= 1 << 21
    assert tile(es.OP_SORT_PAIRS, es.INT32, 8) == ((768, 16) if mid else (768, 12) if small else (512, 24))
    assert tile(es.OP_ARGSORT, es.INT32, 8) == tile(es.OP_SORT_PAIRS, es.INT32, 8)
    assert tile(es.OP_SORT_PAIRS, es.INT64, 4) == ((768, 16) if mid else (768, 12) if small else (512, 24))
    assert tile(es.OP_SORT_PAIRS, es.INT64, 8) == ((768, 12) if mid or small else (512, 16))
    assert tile(es.OP_SORT, es.INT64, 0) == (768, 12)
