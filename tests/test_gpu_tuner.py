"""GA autotuner on the GPU: every candidate the search times sorts to the same bytes, and the tuned
parameters sort every distribution exactly as the oracle does (Sec. 3.2, Algorithm 2; Algorithm 1's
check of the tuned sort against a reference)."""
import numpy as np
import pytest

import oracle
import workloads
from gpu_util import assert_bits_equal, require_gpu, to_dev, to_np

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dist", ["uniform", "sorted", "distinct16", "zipf"])
def test_tuned_sort_matches_oracle(dist):
    es = require_gpu()
    from paper_2505_18681_amd import tuner

    n = 300_000
    keys = workloads.make(dist, np.int32, n, 42)
    want = keys[oracle.stable_perm(keys)]
    entry = tuner.tune_sort(es, to_dev(keys), seed=1, pop_size=6, generations=3, reps=1)
    assert entry["evaluations"] >= 6 and len(entry["history"]) == 3
    best = [h["best"] for h in entry["history"]]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:]))
    d = dict(entry["params"])
    d["shape"] = tuple(d["shape"])
    got = to_np(es.sort(to_dev(keys), params=tuner.to_params(es, d)))
    assert_bits_equal(got, want, f"tuned sort {dist} {entry['params']}")


def test_every_candidate_gives_the_same_bytes():
    """The fitness function compares each candidate's output with the first one's; a random
    population over all genes (both routines, every digit width, shapes, thresholds) must pass."""
    es = require_gpu()
    from paper_2505_18681_amd import tuner

    keys = workloads.make("gaussian", np.int64, 200_000, 3)
    dk = to_dev(keys)
    fit = tuner.SortFitness(es, dk, reps=1)
    space = tuner.sort_space()
    repair = tuner.sort_repair(es, es.OP_SORT, es.INT64, keys.size)
    rng = np.random.default_rng(11)
    for _ in range(24):
        fit(repair(space.random(rng, initial=False)))
    assert_bits_equal(to_np(fit.out), keys[oracle.stable_perm(keys)], "last candidate")


def test_tuned_segmented_matches_oracle():
    es = require_gpu()
    from paper_2505_18681_amd import tuner

    sizes = workloads.segment_sizes(3000, 5, median=300.0, sigma=2.0, lo=1, hi=200_000)
    offs = workloads.segment_offsets(sizes)
    keys = workloads.uniform(np.uint32, int(offs[-1]), 5)
    entry = tuner.tune_segmented(es, to_dev(keys), to_dev(offs), seed=2, pop_size=6, generations=2, reps=1)
    d = dict(entry["params"])
    d["shape"] = tuple(d["shape"])
    p = tuner.to_params(es, d)
    got = to_np(es.segmented_sort(to_dev(keys), to_dev(offs), params=p))
    assert_bits_equal(got, oracle.segmented_sort(keys, offs), f"tuned segmented {entry['params']}")


def _keys(dt, n):
    keys = workloads.float_mix(dt, n, 3) if np.dtype(dt).kind == "f" else workloads.uniform(dt, n, 3)
    keys[::11] = keys[5]
    return keys


def test_auto_table_rows_sort_like_the_oracle():
    """Every row of the compiled GA table, taken by EVOSORT_ALGO_AUTO at both ends of its length range and at a
    ragged length inside it, sorts element by element like the oracle through the mergesort (lengths the small
    branch takes first aside)."""
    es = require_gpu()
    from paper_2505_18681_amd import tuner

    rows = tuner.auto_table_rows(tuner.packaged_table())
    assert rows, "the packaged table has rows"
    for name, n, lo, hi, algo in rows:
        dt = np.dtype(name)
        for m in (lo, n + 12_347 if n + 12_347 < hi else n + 7, hi - 1):
            keys = _keys(dt, m)
            k = to_dev(keys)
            auto = es.default_params()
            info = es.plan(es.OP_SORT, es.dtype_code(k.dtype), m, 0, auto)
            small = m < auto.fallback_threshold and m <= info["small_capacity"]  # Algorithm 6's first branch
            assert info["path_name"] == ("small" if small else "merge"), (n, m)
            assert_bits_equal(to_np(es.sort(k, params=auto, check=True)), oracle.sort(keys),
                              f"auto, row at {n}, {m} keys")


@pytest.mark.parametrize("n", [1_000_000 + 4_099, 10_000_000 + 12_347])
@pytest.mark.parametrize("dt", [np.int32, np.float32, np.int64, np.float64])
def test_closed_form_sorts_match_oracle(dt, n):
    """The closed-form parameters (the quadratic refit of the GA's tile picks) sort like the oracle at ragged
    lengths."""
    es = require_gpu()
    from paper_2505_18681_amd import tuner

    keys = _keys(dt, n)
    k = to_dev(keys)
    p = tuner.closed_form_params(es, np.dtype(dt).name, n)
    assert es.plan(es.OP_SORT, es.dtype_code(k.dtype), n, 0, p)["path_name"] == "radix"
    assert_bits_equal(to_np(es.sort(k, params=p, check=True)), oracle.sort(keys), "closed form")
