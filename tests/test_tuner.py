"""GA autotuner (Sec. 3.2, Algorithm 2) on the host: operators, schedule, elitism, search quality.

The fitness functions here are synthetic (no GPU): a separable cost with a
known optimum, so that a plausible mistake in selection, crossover, mutation
or elitism shows up as a worse result or a broken invariant.
"""
import math

import numpy as np
import pytest

from paper_2505_18681_amd import tuner


def synthetic_cost(d: dict) -> float:
    # optimum: algo 4, T_ins 300, T_numpy 50000, d = 8, shape (512, 24)
    return (5.0 * (d["algo"] != 4) + abs(math.log2(d["insertion_threshold"]) - math.log2(300))
            + abs(d["fallback_threshold"] - 50000) / 20000.0 + 1.0 * (d["digit_bits"] != 8)
            + 1.0 * (tuple(d["shape"]) != (512, 24)))


def run_synthetic(seed=42, **kw):
    space = tuner.sort_space()
    calls = []

    def f(ind):
        calls.append(ind)
        return synthetic_cost(space.as_dict(ind))

    return tuner.run_ga(space, f, seed=seed, **kw), calls, space


def test_schedule_is_the_papers():
    """Algorithm 2: 30 individuals, generations 0..9; Sec. 3.2: crossover 0.7, mutation 0.3."""
    assert (tuner.POP_SIZE, tuner.GENERATIONS, tuner.P_CROSSOVER, tuner.P_MUTATION) == (30, 10, 0.7, 0.3)
    res, calls, _ = run_synthetic()
    assert [h["generation"] for h in res.history] == list(range(10))
    assert res.evaluations == len(calls) == len(set(calls))  # each distinct individual timed once


def test_initial_and_full_bounds():
    """Generation 0 draws T_ins in [2, 256] and T_numpy in [30000, 100000]; later draws use [2, 2048], [1000, 100000]."""
    space = tuner.sort_space()
    rng = np.random.default_rng(0)
    init = [space.as_dict(space.random(rng, initial=True)) for _ in range(2000)]
    full = [space.as_dict(space.random(rng, initial=False)) for _ in range(2000)]
    assert min(d["insertion_threshold"] for d in init) >= 2 and max(d["insertion_threshold"] for d in init) <= 256
    assert min(d["fallback_threshold"] for d in init) >= 30000
    assert max(d["fallback_threshold"] for d in init) <= 100000
    assert max(d["insertion_threshold"] for d in full) > 256  # the wider bounds are used
    assert min(d["fallback_threshold"] for d in full) < 30000
    assert all(space.contains(space.random(rng, initial=False)) for _ in range(500))
    assert {d["algo"] for d in init} == {3, 4}


def test_elitism_keeps_the_best():
    res, _, _ = run_synthetic()
    best = [h["best"] for h in res.history]
    assert all(b2 <= b1 for b1, b2 in zip(best, best[1:])), best
    assert res.best_fitness == best[-1]


def test_search_finds_the_optimum_region():
    res, _, space = run_synthetic()
    d = res.best_dict()
    assert d["algo"] == 4 and d["digit_bits"] == 8 and tuple(d["shape"]) == (512, 24)
    assert res.best_fitness < 1.0
    # better than the best of generation 0 and far better than its mean
    assert res.best_fitness < res.history[0]["best"] and res.best_fitness < 0.25 * res.history[0]["mean"]


def test_ga_beats_random_search_of_equal_budget():
    res, calls, space = run_synthetic(seed=7)
    rng = np.random.default_rng(7)
    rand = min(synthetic_cost(space.as_dict(space.random(rng, initial=False))) for _ in range(len(calls)))
    assert res.best_fitness <= rand


def test_deterministic_for_a_seed():
    a, _, _ = run_synthetic(seed=3)
    b, _, _ = run_synthetic(seed=3)
    c, _, _ = run_synthetic(seed=4)
    assert a.best == b.best and a.history == b.history
    assert a.history != c.history


def test_uniform_crossover_keeps_genes_in_place():
    rng = np.random.default_rng(1)
    a, b = (1, 2, 3, 4, 5), (10, 20, 30, 40, 50)
    swaps = 0
    for _ in range(200):
        c, d = tuner.uniform_crossover(a, b, rng)
        for i in range(5):
            assert {c[i], d[i]} == {a[i], b[i]}
        swaps += sum(ci != ai for ci, ai in zip(c, a))
    assert 350 < swaps < 650  # about half of 1000 positions


def test_uniform_mutation_rate_and_bounds():
    space = tuner.sort_space()
    rng = np.random.default_rng(2)
    ind = (4, 300, 50000, 8, (512, 24))
    assert tuner.uniform_mutation(ind, space, rng, 0.0) == ind
    changed = 0
    for _ in range(400):
        m = tuner.uniform_mutation(ind, space, rng, 0.3)
        assert space.contains(m)
        changed += sum(x != y for x, y in zip(m, ind))
    # 0.3 per gene, minus redraws that land on the same value (choices of 2..12 options)
    assert 300 < changed < 640


def test_tournament_prefers_fitter():
    rng = np.random.default_rng(3)
    pop = [(i,) for i in range(30)]
    fit = {p: float(p[0]) for p in pop}
    picks = [tuner.tournament(pop, fit, rng, 3)[0] for _ in range(3000)]
    assert np.mean(picks) < 10  # size-3 tournaments: expected rank about 7 of 30
    assert min(picks) == 0


def test_seed_individual_survives_when_best():
    space = tuner.sort_space()
    opt = (4, 300, 50000, 8, (512, 24))
    res = tuner.run_ga(space, lambda ind: synthetic_cost(space.as_dict(ind)), seed=1, pop_size=8, generations=3,
                       seed_individuals=[opt])
    assert res.best == opt and res.best_fitness == 0.0


def test_repair_through_the_library_plan():
    """Shapes not compiled at a digit width fall back to the default shape (host-only plan call)."""
    es = pytest.importorskip("paper_2505_18681_amd")
    repair = tuner.sort_repair(es, es.OP_SORT, es.INT32, 10 ** 6)
    space = tuner.sort_space()
    rng = np.random.default_rng(5)
    for _ in range(200):
        ind = repair(space.random(rng, initial=False))
        es.plan(es.OP_SORT, es.INT32, 10 ** 6, 0, tuner.to_params(es, space.as_dict(ind)))  # raises if invalid
    # an alternative shape exists only at 8-bit digits
    fixed = space.as_dict(repair((4, 8, 50000, 11, (256, 48))))
    assert fixed["digit_bits"] == 11 and tuple(fixed["shape"]) == (0, 0)


def test_params_for_picks_the_nearest_size_class():
    es = pytest.importorskip("paper_2505_18681_amd")
    table = {"entries": [
        {"dtype": "int32", "dist": "uniform", "n": 10 ** 6, "params": {"algo": 4, "digit_bits": 8,
                                                                        "shape": [512, 16]}},
        {"dtype": "int32", "dist": "uniform", "n": 10 ** 8, "params": {"algo": 4, "digit_bits": 8,
                                                                        "shape": [512, 24]}},
        {"dtype": "int32", "dist": "sorted", "n": 10 ** 8, "params": {"algo": 3, "insertion_threshold": 64}},
    ]}
    p = tuner.params_for(es, table, "int32", 3 * 10 ** 7)
    assert (p.block_threads, p.items_per_thread) == (512, 24)
    p = tuner.params_for(es, table, "int32", 2 * 10 ** 6)
    assert (p.block_threads, p.items_per_thread) == (512, 16)
    p = tuner.params_for(es, table, "int32", 10 ** 8, "sorted")
    assert p.algo == 3 and p.insertion_threshold == 64
    p = tuner.params_for(es, table, "int64", 10 ** 8)
    d = es.default_params()
    assert (p.algo, p.digit_bits) == (d.algo, d.digit_bits)


# --------------------------------------------------------------------------
# Closed forms (Sec. 7, Eq. 1 and Eq. 2) and the table the library compiles in
# --------------------------------------------------------------------------
def test_paper_closed_forms_match_worked_values(golden):
    from paper_2505_18681_amd import tuner

    rows = golden("paper_closed_form.txt")
    assert len(rows) == 4
    for n, t_ins, t_np in rows:
        assert tuner.paper_thresholds(int(n)) == (int(t_ins), int(t_np)), n


def test_paper_closed_forms_have_the_stated_extrema():
    """Sec. 7 states the extrema x* = -b / (2a): about 8.17 for T_insertion and 6.45 for T_numpy."""
    from paper_2505_18681_amd import tuner

    for coeffs, x_star in ((tuner.PAPER_T_INSERTION, 8.17), (tuner.PAPER_T_NUMPY, 6.45)):
        a, b, _ = coeffs
        assert a < 0 and abs(-b / (2 * a) - x_star) < 0.01


def test_gpu_tile_formula_refits_from_the_table():
    """The committed coefficients are the least-squares fit over the packaged GA table."""
    es = pytest.importorskip("paper_2505_18681_amd")
    from paper_2505_18681_amd import tuner

    table = tuner.packaged_table()
    for kb in (4, 8):
        fit = tuner.fit_tile_formula(es, table, kb)
        assert all(abs(f - c) < 1e-3 for f, c in zip(fit, tuner.GPU_TILE_FORMULA[kb])), (kb, fit)


def test_gpu_tile_formula_tracks_the_tables_picks():
    """At every size class the GA tuned with the radix routine, the closed form's tile is within a factor of
    two of the GA's pick (shapes exist only in steps)."""
    import math

    es = pytest.importorskip("paper_2505_18681_amd")
    from paper_2505_18681_amd import tuner

    checked = 0
    for e in tuner.packaged_table()["entries"]:
        if e["dist"] != "uniform":
            continue
        d = dict(e["params"])
        d["shape"] = tuple(d["shape"])
        pick = tuner.effective_tile(es, e["dtype"], e["n"], tuner.to_params(es, d))
        if not pick:
            continue
        form = tuner.effective_tile(es, e["dtype"], e["n"], tuner.closed_form_params(es, e["dtype"], e["n"]))
        assert abs(math.log2(form) - math.log2(pick)) <= 1.0, (e["dtype"], e["n"], form, pick)
        checked += 1
    assert checked >= 10


def test_compiled_table_is_the_packaged_one():
    """csrc/tuned_table.hpp is what the emitter writes for the packaged GA table."""
    from paper_2505_18681_amd import tuner

    with open(tuner.HEADER_PATH) as f:
        assert f.read() == tuner.emit_header(tuner.packaged_table())


def test_auto_dispatch_follows_the_table():
    """EVOSORT_ALGO_AUTO of a keys-only sort takes a row's routine (the mergesort) for every length in the row's
    range and nowhere outside it; explicit A_code 4, a given shape, pairs and argsort keep the radix sort."""
    es = pytest.importorskip("paper_2505_18681_amd")
    from paper_2505_18681_amd import tuner

    rows = tuner.auto_table_rows(tuner.packaged_table())
    assert rows, "the packaged table has rows"
    for dt, n, lo, hi, algo in rows:
        assert lo <= n < hi and algo == es.ALGO_MERGE
        code = tuner.DTYPE_CODES[dt]
        for m in (lo, n, hi - 1):
            info = es.plan(es.OP_SORT, code, m)
            if m < es.default_params().fallback_threshold and m <= info["small_capacity"]:
                assert info["path_name"] == "small", (dt, m)  # Algorithm 6 takes the small branch first
                continue
            assert info["path_name"] == "merge", (dt, m)
            assert es.plan(es.OP_SORT, code, m, 0, es.default_params(algo=es.ALGO_RADIX))["path_name"] == "radix"
            assert es.plan(es.OP_SORT_PAIRS, code, m, 4)["path_name"] == "radix"
            assert es.plan(es.OP_ARGSORT, code, m, 4)["path_name"] == "radix"
            given = es.plan(es.OP_SORT, code, m, 0, es.default_params(block_threads=512, items_per_thread=16))
            assert (given["path_name"], given["block_threads"], given["items_per_thread"]) == ("radix", 512, 16)
        for m in (lo - 1, hi):
            if any(r[0] == dt and r[2] <= m < r[3] for r in rows):
                continue
            assert es.plan(es.OP_SORT, code, m)["path_name"] in ("radix", "small", "copy"), (dt, m)


def test_auto_table_row_ranges_tile_the_size_classes():
    """A row's range runs from the geometric mean with the next smaller tuned size class of its key type to the
    one with the next larger (half a decade past the ends); only mergesort picks that pass the gain bar, agreed
    on by every entry of their class, give rows."""
    from paper_2505_18681_amd import tuner

    def entry(dtype, n, algo, shape, ms, default_ms):
        return {"dtype": dtype, "dist": "uniform", "n": n, "ms": ms, "default_ms": default_ms,
                "params": {"algo": algo, "shape": list(shape), "digit_bits": 8}}

    table = {"entries": [
        entry("int64", 10_000, 4, (0, 0), 1.0, 1.0),
        entry("int64", 20_000, 3, (512, 8), 0.8, 1.0),          # the mergesort: its shape gene is moot
        entry("float64", 20_000, 3, (1024, 16), 0.8, 1.0),      # the only float64 class
        entry("int64", 50_000, 3, (0, 0), 0.8, 1.0),
        entry("int64", 50_000, 4, (0, 0), 1.0, 1.0),            # a second run of the class disagrees
        entry("int64", 100_000, 4, (512, 16), 0.9, 1.0),        # a radix tile pick: no row
        entry("int64", 200_000, 3, (0, 0), 0.96, 1.0),          # gain below the 5 % bar
        entry("int32", 1_000_000, 3, (0, 0), 0.9, 1.0),
        entry("int32", 1_000_000, 4, (0, 0), 0.9, 1.0) | {"dist": "zipf"},
    ]}
    rows = tuner.auto_table_rows(table)
    assert rows == [("int32", 1_000_000, 316_228, 3_162_278, 3),
                    ("int64", 20_000, 14_143, 31_623, 3),
                    ("float64", 20_000, 6_325, 63_246, 3)]
    # each bound is the smallest length at or above the geometric mean
    assert 14_142 ** 2 < 10_000 * 20_000 <= 14_143 ** 2
    assert 31_622 ** 2 < 20_000 * 50_000 <= 31_623 ** 2
    assert 10 * 316_227 ** 2 < 10 ** 12 <= 10 * 316_228 ** 2
    assert 10 * 6_324 ** 2 < 20_000 ** 2 <= 10 * 6_325 ** 2
    header = tuner.emit_header(table)
    assert "    {2, 20000, 14143, 31623, 3},  // int64" in header
    assert "constexpr int kTunedRowCount = 3;" in header


def test_retime_pair_alternates_and_takes_medians():
    """The re-timing after the search alternates the two settings, so a clock that speeds up over the
    re-timing favours neither; each side's figure is the median of its own timings."""
    from paper_2505_18681_amd import tuner

    order, clock = [], iter(range(100, 0, -1))  # every timing faster than the one before

    def timer(tag):
        def f():
            order.append(tag)
            return float(next(clock))
        return f

    a, b = tuner.retime_pair(timer("a"), timer("b"), rounds=5)
    assert order == ["a", "b"] * 5
    assert (a, b) == (96.0, 95.0)  # medians of 100, 98, 96, 94, 92 and of 99, 97, 95, 93, 91
    assert tuner.RETIME_ROUNDS >= 5
