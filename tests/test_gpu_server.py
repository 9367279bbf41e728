"""Sort server on the GPU: every result of a mixed, overlapping, batched request stream equals the oracle's
stable sort of that request and the same request sorted alone (bit for bit; the stable sort is unique),
the HBM budget holds, results copied out and released without a synchronization stay intact, and a job
whose kernels fail is reported as failed."""
import time

import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu

DTYPES = (np.int32, np.int64, np.float32, np.uint32, np.float64)


def make_requests(count, seed, lo=1, hi=300_000):
    rng = np.random.default_rng(seed)
    sizes = np.exp(rng.uniform(np.log(lo), np.log(hi), size=count)).astype(np.int64)
    out = []
    for i, n in enumerate(sizes):
        dt = DTYPES[int(rng.integers(len(DTYPES)))]
        if dt in (np.float32, np.float64):
            keys = workloads.float_mix(dt, int(n), seed * 1000 + i)
        else:
            keys = workloads.uniform(dt, int(n), seed * 1000 + i)
        if i % 7 == 3:
            keys[: n // 2] = keys[0]  # runs of equal keys
        out.append(keys)
    return out


def test_mixed_stream_matches_each_request_alone():
    es = require_gpu()
    reqs = make_requests(240, 1)
    dev = [to_dev(k) for k in reqs]
    with es.Server(hbm_budget_bytes=1 << 30, streams=4, batch_max_keys=20_000) as srv:
        ids = []
        rng = np.random.default_rng(2)
        for d in dev:
            ids.append(srv.submit(d))
            if rng.random() < 0.2:
                time.sleep(0.0005)  # arrivals while earlier work runs
        for i, (rid, keys, d) in enumerate(zip(ids, reqs, dev)):
            got = to_np(srv.result(rid))
            assert_bits_equal(got, keys[oracle.stable_perm(keys)], f"request {i} (n={keys.size}, {keys.dtype}) "
                                                                   "vs oracle")
            alone = to_np(es.sort(d))
            assert_bits_equal(got, alone, f"request {i} vs alone")
            srv.release(rid)
        st = srv.stats()
    assert st["completed"] == st["submitted"] == len(reqs) and st["failed"] == 0
    assert st["batched_requests"] > 0, st
    assert st["jobs"] < len(reqs), st  # short requests shared launches
    assert st["max_concurrent_jobs"] >= 2, st
    assert st["bytes_in_use"] == 0 and st["released"] == len(reqs)


def test_budget_bounds_the_arena_and_every_request_finishes():
    es = require_gpu()
    rng = np.random.default_rng(3)
    reqs = [workloads.uniform(np.int32, int(n), 40 + i) for i, n in enumerate(rng.integers(200_000, 1_500_000, 40))]
    dev = [to_dev(k) for k in reqs]
    budget = 64 << 20  # a few requests at a time
    with es.Server(hbm_budget_bytes=budget, streams=4, batch_max_keys=0) as srv:
        ids = [srv.submit(d) for d in dev]
        for rid, keys in zip(ids, reqs):
            got = to_np(srv.result(rid))
            assert_bits_equal(got, oracle.sort(keys), "budgeted request")
            srv.release(rid)
        st = srv.stats()
    assert st["peak_bytes"] <= budget and st["completed"] == len(reqs)
    assert st["batched_requests"] == 0


def test_over_budget_request_is_refused():
    es = require_gpu()
    with es.Server(hbm_budget_bytes=8 << 20, streams=2) as srv:
        big = to_dev(workloads.uniform(np.int64, 2_000_000, 5))
        with pytest.raises(es.EvosortError) as e:
            srv.submit(big)
        assert e.value.status == es.ERR_OVER_BUDGET
        small = workloads.uniform(np.int64, 1000, 6)
        rid = srv.submit(to_dev(small))
        assert_bits_equal(to_np(srv.result(rid)), oracle.sort(small), "small after refusal")


def test_unreleased_results_hold_memory_until_release():
    es = require_gpu()
    reqs = [workloads.uniform(np.float32, 100_000 + i, 70 + i) for i in range(6)]
    with es.Server(hbm_budget_bytes=256 << 20, streams=2, batch_max_keys=0) as srv:
        ids = [srv.submit(to_dev(k)) for k in reqs]
        srv.drain()
        assert srv.stats()["bytes_in_use"] > 0
        for rid in ids:
            assert srv.done(rid)
            srv.release(rid)
        assert srv.stats()["bytes_in_use"] == 0


def test_one_stream_runs_one_job_at_a_time():
    es = require_gpu()
    reqs = make_requests(30, 9, lo=1000, hi=200_000)
    with es.Server(hbm_budget_bytes=512 << 20, streams=1, batch_max_keys=0) as srv:
        ids = [srv.submit(to_dev(k)) for k in reqs]
        for rid, keys in zip(ids, reqs):
            assert_bits_equal(to_np(srv.result(rid)), keys[oracle.stable_perm(keys)], "one stream")
            srv.release(rid)
        st = srv.stats()
    assert st["max_concurrent_jobs"] == 1 and st["jobs"] == len(reqs)


def test_empty_request():
    es = require_gpu()
    import torch

    with es.Server(hbm_budget_bytes=16 << 20) as srv:
        rid = srv.submit(torch.empty(0, dtype=torch.int32, device="cuda"))
        assert srv.done(rid)
        assert srv.result(rid).numel() == 0
        srv.release(rid)


def test_result_then_release_without_synchronizing():
    """result() queues a copy on the client's stream and release() returns the arena range at once; the
    range must not be handed to a later job before that copy has run.  New requests are admitted into the
    freed memory while the copies may still be queued; every copied result is checked against the oracle
    after one final synchronization."""
    es = require_gpu()
    import torch

    reqs = [workloads.uniform(np.int64, int(n), 90 + i)
            for i, n in enumerate(np.random.default_rng(4).integers(100_000, 900_000, 48))]
    dev = [to_dev(k) for k in reqs]
    stream = torch.cuda.current_stream()
    copies = []
    # a small budget: few requests fit at once, so admission reuses released ranges right away
    with es.Server(hbm_budget_bytes=48 << 20, streams=4, batch_max_keys=0) as srv:
        ids = [srv.submit(d) for d in dev[:8]]
        nxt = 8
        while ids:
            rid = ids.pop(0)
            srv.wait(rid)
            # keep the client stream busy so the copy below is still queued when release() runs
            torch.cuda._sleep(2_000_000)
            copies.append(srv.result(rid))
            srv.release(rid)
            if nxt < len(dev):
                ids.append(srv.submit(dev[nxt]))
                nxt += 1
        stream.synchronize()
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    for i, (got, keys) in enumerate(zip(copies, reqs)):
        assert_bits_equal(to_np(got), oracle.sort(keys), f"copied result {i}")


def test_failed_job_is_reported_not_ok():
    """A served sort whose look-back wait runs out (a debug switch withholds tile 0's counts) finishes with
    EVOSORT_ERR_DEVICE_TIMEOUT; the failure stays with the server and the next sorts run normally."""
    es = require_gpu()
    bad = es.default_params(fallback_threshold=0, spin_limit=2000, debug_flags=es.DEBUG_WITHHOLD_TILE0)
    keys = workloads.uniform(np.int32, 60_000, 12)
    with es.Server(hbm_budget_bytes=64 << 20, streams=2, batch_max_keys=0, params=bad) as srv:
        rid = srv.submit(to_dev(keys))
        with pytest.raises(es.EvosortError) as e:
            srv.wait(rid)
        assert e.value.status == es.ERR_DEVICE_TIMEOUT
        assert srv.stats()["failed"] == 1
        srv.release(rid)
    # the server's failure is not charged to the library's next public call
    assert_bits_equal(to_np(es.sort(to_dev(keys), check=True)), oracle.sort(keys), "after a failed job")
    good = es.default_params(fallback_threshold=0)
    with es.Server(hbm_budget_bytes=64 << 20, streams=2, batch_max_keys=0, params=good) as srv:
        rid = srv.submit(to_dev(keys))
        assert_bits_equal(to_np(srv.result(rid)), oracle.sort(keys), "good server")
