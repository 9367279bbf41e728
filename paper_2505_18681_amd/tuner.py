"""Genetic-algorithm autotuner for the GPU sort's parameters.

This is the paper's GA driver (Sec. 3.2, the parameter vector and the
fitness f(x) = T_sort(x); Algorithm 2, RunGATuning) retargeted from the CPU
routine's three parameters to the parameters of this library:

    algo                 A_code: 3 mergesort, 4 LSD radix sort
    insertion_threshold  T_insertion: mergesort chunk length
    fallback_threshold   T_numpy: one-workgroup sort below this length
    digit_bits           radix digit width d
    shape                radix tile shape (threads, keys per thread)

The GA follows the paper's schedule: a population of 30 over 10 generations;
generation 0 drawn from the narrower initial bounds (T_insertion in [2, 256],
T_numpy in [30000, 100000]) and later generations from the full bounds
(T_insertion in [2, 2048], T_numpy in [1000, 100000]); each generation keeps
its best individuals unchanged (elitism), breeds the rest by uniform
crossover with probability 0.7 and uniform mutation with probability 0.3,
and re-times only the individuals that crossover or mutation changed.  The
paper leaves the parent selection, the number of elites and the exact
meaning of the mutation probability open; the readings used here are
tournament selection of size 3, two elites, and a per-gene probability of
0.3 of redrawing the gene uniformly from its bounds.

Every parameter setting produces the same bytes (the stable sort is
unique), so the GA changes speed only; the GPU fitness function checks each
candidate's output against the first candidate's, bit for bit.

The GA core (`GeneSpace`, `run_ga`) is plain Python and runs without a GPU;
`SortFitness`, `SegmentedFitness`, `tune_sort` and `tune_segmented` time the
library's sorts on the current GPU.
"""
from __future__ import annotations

import dataclasses
import json
import math
import time
from typing import Callable, Dict, List, Optional, Sequence, Tuple

import numpy as np

POP_SIZE = 30        # Algorithm 2: 30 individuals
GENERATIONS = 10     # Algorithm 2: generations 0..9
P_CROSSOVER = 0.7    # Sec. 3.2: uniform crossover probability
P_MUTATION = 0.3     # Sec. 3.2: uniform mutation probability
TOURNAMENT = 3       # reading: parent selection (the paper does not name one)
ELITES = 2           # reading: individuals kept unchanged per generation


@dataclasses.dataclass(frozen=True)
class Gene:
    """One parameter: an integer range (lo..hi, inclusive) or a list of choices.

    lo0/hi0 bound the integer draw of generation 0 (the paper's initial
    bounds); later draws use lo/hi.  Choices are drawn uniformly in every
    generation.
    """

    name: str
    lo: int = 0
    hi: int = 0
    lo0: Optional[int] = None
    hi0: Optional[int] = None
    choices: Optional[Tuple] = None

    def draw(self, rng: np.random.Generator, initial: bool):
        if self.choices is not None:
            return self.choices[int(rng.integers(len(self.choices)))]
        lo = self.lo0 if (initial and self.lo0 is not None) else self.lo
        hi = self.hi0 if (initial and self.hi0 is not None) else self.hi
        return int(rng.integers(lo, hi + 1))

    def contains(self, value) -> bool:
        if self.choices is not None:
            return value in self.choices
        return isinstance(value, (int, np.integer)) and self.lo <= int(value) <= self.hi


class GeneSpace:
    """The genome layout: an ordered list of genes; an individual is a tuple of values."""

    def __init__(self, genes: Sequence[Gene]):
        self.genes = list(genes)
        self.names = [g.name for g in self.genes]

    def random(self, rng: np.random.Generator, initial: bool) -> tuple:
        return tuple(g.draw(rng, initial) for g in self.genes)

    def contains(self, ind: tuple) -> bool:
        return len(ind) == len(self.genes) and all(g.contains(v) for g, v in zip(self.genes, ind))

    def as_dict(self, ind: tuple) -> dict:
        return dict(zip(self.names, ind))


def uniform_crossover(a: tuple, b: tuple, rng: np.random.Generator) -> Tuple[tuple, tuple]:
    """Each gene position is exchanged between the two parents with probability 1/2."""
    swap = rng.random(len(a)) < 0.5
    c = tuple(y if s else x for x, y, s in zip(a, b, swap))
    d = tuple(x if s else y for x, y, s in zip(a, b, swap))
    return c, d


def uniform_mutation(ind: tuple, space: GeneSpace, rng: np.random.Generator, p_gene: float) -> tuple:
    """Each gene is redrawn uniformly from its full bounds with probability p_gene."""
    return tuple(g.draw(rng, initial=False) if rng.random() < p_gene else v for g, v in zip(space.genes, ind))


def tournament(pop: List[tuple], fit: Dict[tuple, float], rng: np.random.Generator, k: int) -> tuple:
    """The fittest (lowest time) of k individuals drawn uniformly with replacement."""
    picks = [pop[int(i)] for i in rng.integers(len(pop), size=k)]
    return min(picks, key=lambda x: fit[x])


@dataclasses.dataclass
class GAResult:
    best: tuple
    best_fitness: float
    history: List[dict]          # per generation: best, mean, worst fitness and evaluations so far
    evaluations: int             # distinct individuals timed
    space: GeneSpace

    def best_dict(self) -> dict:
        return self.space.as_dict(self.best)


def run_ga(space: GeneSpace, fitness: Callable[[tuple], float], *, seed: int = 42, pop_size: int = POP_SIZE,
           generations: int = GENERATIONS, p_crossover: float = P_CROSSOVER, p_mutation: float = P_MUTATION,
           tournament_size: int = TOURNAMENT, elites: int = ELITES,
           repair: Optional[Callable[[tuple], tuple]] = None,
           seed_individuals: Sequence[tuple] = ()) -> GAResult:
    """RunGATuning (Algorithm 2): minimise `fitness` over `space`.

    `repair` maps any individual to a valid one (e.g. a tile shape that is not
    compiled at a digit width); `seed_individuals` are placed in generation 0
    before the random draws (the library's defaults, so the result is never
    slower than them up to timing noise).  Fitness values are cached per
    distinct individual: an individual that survives unchanged is not re-timed.
    """
    if pop_size < 2 or generations < 1:
        raise ValueError("pop_size >= 2 and generations >= 1 are required")
    rng = np.random.default_rng(seed)
    fix = repair or (lambda x: x)
    fit: Dict[tuple, float] = {}

    def evaluate(pop):
        for ind in pop:
            if ind not in fit:
                fit[ind] = float(fitness(ind))

    # Generation 0: initial bounds
    pop = [fix(tuple(s)) for s in seed_individuals][:pop_size]
    while len(pop) < pop_size:
        pop.append(fix(space.random(rng, initial=True)))
    history = []
    n_elite = min(elites, pop_size - 1)
    for g in range(generations):
        evaluate(pop)  # fitness of every individual (cached ones are not re-timed)
        vals = [fit[x] for x in pop]
        history.append({"generation": g, "best": min(vals), "mean": float(np.mean(vals)), "worst": max(vals),
                        "evaluations": len(fit)})
        if g == generations - 1:
            break
        ranked = sorted(pop, key=lambda x: fit[x])
        nxt = ranked[:n_elite]  # elitism
        while len(nxt) < pop_size:
            a = tournament(pop, fit, rng, tournament_size)
            b = tournament(pop, fit, rng, tournament_size)
            if rng.random() < p_crossover:
                a, b = uniform_crossover(a, b, rng)
            a = uniform_mutation(a, space, rng, p_mutation)
            b = uniform_mutation(b, space, rng, p_mutation)
            nxt.append(fix(a))
            if len(nxt) < pop_size:
                nxt.append(fix(b))
        pop = nxt
    best = min(pop, key=lambda x: fit[x])
    return GAResult(best=best, best_fitness=fit[best], history=history, evaluations=len(fit), space=space)


# --------------------------------------------------------------------------
# The library's parameter space
# --------------------------------------------------------------------------
# Radix tile shapes (threads, keys per thread); (0, 0) = the library default.
# Which of them are compiled at a given digit width is asked of evosort_plan.
RADIX_SHAPES = ((0, 0), (256, 8), (256, 12), (256, 16), (256, 24), (256, 32), (256, 48), (512, 8), (512, 16),
                (512, 24), (512, 32), (768, 12), (768, 16), (768, 20), (768, 24), (1024, 8), (1024, 12), (1024, 16),
                (1024, 20))
SEG_SHAPES = ((0, 0), (512, 24), (768, 24), (768, 12), (1024, 16), (512, 16), (256, 16), (256, 8))


def sort_space() -> GeneSpace:
    """Genome of one sort call: (algo, T_insertion, T_numpy, digit_bits, shape)."""
    return GeneSpace([
        Gene("algo", choices=(3, 4)),
        Gene("insertion_threshold", lo=2, hi=2048, lo0=2, hi0=256),
        Gene("fallback_threshold", lo=1000, hi=100000, lo0=30000, hi0=100000),
        Gene("digit_bits", choices=(4, 5, 6, 7, 8, 9, 10, 11, 12)),
        Gene("shape", choices=RADIX_SHAPES),
    ])


def segmented_space(capacity: int) -> GeneSpace:
    """Genome of one batched call: (segment length below which one workgroup sorts it, tile shape)."""
    return GeneSpace([
        Gene("fallback_threshold", lo=0, hi=capacity + 1, lo0=capacity // 8, hi0=capacity + 1),
        Gene("shape", choices=SEG_SHAPES),
    ])


def to_params(es, d: dict):
    """Library params (evosort_params) for a genome dict of sort_space / segmented_space."""
    p = es.default_params()
    for k in ("algo", "insertion_threshold", "fallback_threshold", "digit_bits"):
        if k in d:
            setattr(p, k, int(d[k]))
    if "shape" in d:
        p.block_threads, p.items_per_thread = (int(x) for x in d["shape"])
    return p


def sort_repair(es, op: int, dtype_code: int, n: int, value_bytes: int = 0) -> Callable[[tuple], tuple]:
    """Map a sort_space individual to one the library accepts for (op, dtype, n).

    A shape that is not compiled at the digit width falls back to the default
    shape; a digit width that still has no kernel falls back to 8 bits.  The
    check is evosort_plan (host only).
    """
    space = sort_space()

    def ok(ind):
        try:
            es.plan(op, dtype_code, n, value_bytes, to_params(es, space.as_dict(ind)))
            return True
        except es.EvosortError:
            return False

    def repair(ind: tuple) -> tuple:
        d = space.as_dict(ind)
        if ok(ind):
            return ind
        d["shape"] = (0, 0)
        ind2 = tuple(d[k] for k in space.names)
        if ok(ind2):
            return ind2
        d["digit_bits"] = 8
        return tuple(d[k] for k in space.names)

    return repair


# --------------------------------------------------------------------------
# GPU fitness: median wall time of the sort on resident sample data
# --------------------------------------------------------------------------
WARM_SECONDS = 0.25


def _spin(call, torch, seconds: float) -> None:
    """Runs `call` (at least 3 times) until `seconds` of wall time have passed."""
    t0 = time.perf_counter()
    k = 0
    while k < 3 or time.perf_counter() - t0 < seconds:
        call()
        torch.cuda.synchronize()
        k += 1


class SortFitness:
    """f(x) = T_sort(x) (Sec. 3.2): median GPU time of one sort call, in ms.

    The keys stay on the device; each evaluation runs one untimed call, then
    `reps` calls timed with HIP events on the current stream.  The output of
    every candidate is compared bit for bit with the output of the first one
    (all settings must produce the same stable sort); a difference raises.
    """

    def __init__(self, es, keys, *, reps: int = 3, space: Optional[GeneSpace] = None):
        import torch

        self.es, self.torch, self.keys, self.reps = es, torch, keys, reps
        self.space = space or sort_space()
        self.out = torch.empty_like(keys)
        self.reference = None
        self.temp = None
        self.calls = 0
        self.memo: Dict[tuple, float] = {}

    def _temp(self, params):
        es, torch = self.es, self.torch
        need = max(es.temp_bytes(es.OP_SORT, es.dtype_code(self.keys.dtype), self.keys.numel(), 0, params), 256)
        if self.temp is None or self.temp.numel() < need:
            self.temp = None
            self.temp = torch.empty(need, dtype=torch.uint8, device=self.keys.device)
        return self.temp

    def effective_key(self, params) -> tuple:
        """What the call does with these params: genes that the chosen routine ignores are dropped."""
        es = self.es
        info = es.plan(es.OP_SORT, es.dtype_code(self.keys.dtype), self.keys.numel(), 0, params)
        path = info["path_name"]
        if path == "radix":
            return (path, info["digit_bits"], info["block_threads"], info["items_per_thread"])
        if path == "merge":
            return (path, int(params.insertion_threshold))
        return (path,)

    def __call__(self, ind: tuple) -> float:
        es, torch = self.es, self.torch
        p = to_params(es, self.space.as_dict(ind))
        key = self.effective_key(p)
        if key in self.memo:
            return self.memo[key]
        t = self._time(p)
        self.memo[key] = t
        return t

    def warm(self, ind: tuple, seconds: float = WARM_SECONDS) -> None:
        """Untimed sorts with one individual's params before the first timing, so that the
        first individuals timed (the seeded defaults) do not meet an idle GPU's clocks."""
        p = to_params(self.es, self.space.as_dict(ind))
        tmp = self._temp(p)
        _spin(lambda: self.es.sort(self.keys, params=p, out=self.out, temp=tmp), self.torch, seconds)

    def _time(self, p) -> float:
        es, torch = self.es, self.torch
        tmp = self._temp(p)
        es.sort(self.keys, params=p, out=self.out, temp=tmp)
        torch.cuda.synchronize()
        times = []
        stream = torch.cuda.current_stream()
        for _ in range(self.reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            es.sort(self.keys, params=p, out=self.out, temp=tmp)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        self.calls += 1
        bits = self.out.view(torch.uint8)
        if self.reference is None:
            self.reference = bits.clone()
        elif not torch.equal(bits, self.reference):
            raise RuntimeError(f"parameters {p} changed the sorted output")
        return float(np.median(times))


class SegmentedFitness:
    """f(x) = median GPU time of one batched segmented call on a resident batch, in ms."""

    def __init__(self, es, keys, offsets, *, reps: int = 3):
        import torch

        self.es, self.torch, self.keys, self.offsets, self.reps = es, torch, keys, offsets, reps
        self.space = segmented_space(es.segmented_capacity(es.dtype_code(keys.dtype)))
        self.out = torch.empty_like(keys)
        self.reference = None
        self.temp = None

    def _call(self, ind: tuple):
        es, torch = self.es, self.torch
        p = to_params(es, self.space.as_dict(ind))
        code = es.dtype_code(self.keys.dtype)
        need = es.segmented_temp_bytes(code, self.keys.numel(), self.offsets.numel() - 1, 0, p)
        if self.temp is None or self.temp.numel() < need:
            self.temp = None
            self.temp = torch.empty(need, dtype=torch.uint8, device=self.keys.device)
        return lambda: es.segmented_sort(self.keys, self.offsets, params=p, out=self.out, temp=self.temp)  # noqa

    def warm(self, ind: tuple, seconds: float = WARM_SECONDS) -> None:
        """Untimed batched calls with one individual's params before the first timing."""
        _spin(self._call(ind), self.torch, seconds)

    def __call__(self, ind: tuple) -> float:
        torch = self.torch
        call = self._call(ind)
        call()
        torch.cuda.synchronize()
        times = []
        stream = torch.cuda.current_stream()
        for _ in range(self.reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            call()
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b))
        bits = self.out.view(torch.uint8)
        if self.reference is None:
            self.reference = bits.clone()
        elif not torch.equal(bits, self.reference):
            raise RuntimeError(f"parameters {self.space.as_dict(ind)} changed the segmented output")
        return float(np.median(times))


# After the search the default and the GA's pick are timed again, alternately,
# this many times each; the table records the two medians.
RETIME_ROUNDS = 7


def retime_pair(time_a: Callable[[], float], time_b: Callable[[], float], rounds: int = RETIME_ROUNDS):
    """Medians of `rounds` timings of each of two settings taken alternately (a, b, a, b, ...), so that a drift
    of the GPU's clocks during the re-timing falls on both alike rather than on whichever went first."""
    ta, tb = [], []
    for _ in range(rounds):
        ta.append(time_a())
        tb.append(time_b())
    return float(np.median(ta)), float(np.median(tb))


def default_individual(es) -> tuple:
    """The library defaults as a sort_space individual (shape (0, 0) = the default tile shape)."""
    p = es.default_params()
    return (4, int(p.insertion_threshold), min(max(int(p.fallback_threshold), 1000), 100000), int(p.digit_bits),
            (0, 0))


def default_segmented_individual(es, capacity: int) -> tuple:
    """The library defaults as a segmented_space individual."""
    p = es.default_params()
    return (min(int(p.fallback_threshold), capacity + 1), SEG_SHAPES[0])


def tune_sort(es, keys, *, seed: int = 42, pop_size: int = POP_SIZE, generations: int = GENERATIONS,
              reps: int = 3) -> dict:
    """Run the GA for one (dtype, size, distribution) sample held in `keys`; returns a table entry."""
    space = sort_space()
    code = es.dtype_code(keys.dtype)
    fitness = SortFitness(es, keys, reps=reps, space=space)
    repair = sort_repair(es, es.OP_SORT, code, keys.numel())
    base = repair(default_individual(es))
    t0 = time.perf_counter()
    fitness.warm(base)
    res = run_ga(space, fitness, seed=seed, pop_size=pop_size, generations=generations, repair=repair,
                 seed_individuals=[base])
    p_default, p_best = (to_params(es, space.as_dict(x)) for x in (base, res.best))
    default_ms, best_ms = retime_pair(lambda: fitness._time(p_default), lambda: fitness._time(p_best))
    return {"n": int(keys.numel()), "params": _jsonable(res.best_dict()), "ms": round(best_ms, 4),
            "default_ms": round(default_ms, 4), "ga_best_ms": round(res.best_fitness, 4),
            "evaluations": res.evaluations, "history": res.history,
            "search_s": round(time.perf_counter() - t0, 2)}


def tune_segmented(es, keys, offsets, *, seed: int = 42, pop_size: int = POP_SIZE,
                   generations: int = GENERATIONS, reps: int = 3) -> dict:
    """Run the GA for one batch (keys, offsets) of the segmented sort; returns a table entry."""
    fitness = SegmentedFitness(es, keys, offsets, reps=reps)
    cap = es.segmented_capacity(es.dtype_code(keys.dtype))
    base = default_segmented_individual(es, cap)
    t0 = time.perf_counter()
    fitness.warm(base)
    res = run_ga(fitness.space, fitness, seed=seed, pop_size=pop_size, generations=generations,
                 seed_individuals=[base])
    default_ms, best_ms = retime_pair(lambda: fitness(base), lambda: fitness(res.best))
    return {"n": int(keys.numel()), "nseg": int(offsets.numel() - 1), "params": _jsonable(res.best_dict()),
            "ms": round(best_ms, 4), "default_ms": round(default_ms, 4), "ga_best_ms": round(res.best_fitness, 4),
            "evaluations": res.evaluations, "history": res.history,
            "search_s": round(time.perf_counter() - t0, 2)}


def _jsonable(d: dict) -> dict:
    return {k: (list(v) if isinstance(v, tuple) else v) for k, v in d.items()}


def size_class(n: int) -> int:
    """Size classes are decades: 10^k holds lengths in [10^(k-0.5), 10^(k+0.5))."""
    return int(round(math.log10(max(n, 1))))


def params_for(es, table: dict, dtype_name: str, n: int, dist: str = "uniform"):
    """Library params for a sort of n keys from a tuned table: the entry of the same dtype whose
    sample size is nearest to n on a log scale.

    Entries of the requested distribution are preferred, then 'uniform'.
    Returns the library defaults if the table has no entry for the dtype.
    """
    entries = [e for e in table.get("entries", []) if e.get("dtype") == dtype_name]
    for want in (dist, "uniform"):
        cand = [e for e in entries if e.get("dist") == want]
        if cand:
            e = min(cand, key=lambda e: abs(math.log10(max(e["n"], 1)) - math.log10(max(n, 1))))
            d = dict(e["params"])
            if "shape" in d:
                d["shape"] = tuple(d["shape"])
            return to_params(es, d)
    return es.default_params()


def save_table(table: dict, path: str):
    with open(path, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)


def load_table(path: str) -> dict:
    with open(path) as f:
        return json.load(f)


TABLE_PATH = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)),
                                        "tuned", "mi355x.json")


def packaged_table() -> dict:
    """The table this package ships (written by `python -m paper_2505_18681_amd.tuner` on an MI355X), or an
    empty table."""
    import os

    return load_table(TABLE_PATH) if os.path.exists(TABLE_PATH) else {"entries": []}


def tuned_params(es, dtype_name: str, n: int, dist: str = "uniform"):
    """Library params from the packaged table for a sort of n keys (see params_for)."""
    return params_for(es, packaged_table(), dtype_name, n, dist)


# --------------------------------------------------------------------------
# Closed forms (Sec. 7, Eq. 1 and Eq. 2) and the table the library compiles in
# --------------------------------------------------------------------------
# The paper fits each GA-chosen threshold T(n) by a quadratic in x = log10(n)
# and clamps it to the GA's bounds.  Its coefficients, as printed:
PAPER_T_INSERTION = (-106975922 / 731875, 748808234 / 313357, -9314994284 / 997461)
PAPER_T_NUMPY = (-1173315880 / 833461, 15503630602 / 854233, 3935718871 / 743070)


def quadratic(coeffs, n: float) -> float:
    """a x^2 + b x + c at x = log10(n)."""
    a, b, c = coeffs
    x = math.log10(n)
    return a * x * x + b * x + c


def paper_thresholds(n: int) -> Tuple[int, int]:
    """(T_insertion, T_numpy) of the paper's closed forms (Eq. 1, Eq. 2), rounded and clamped to the GA's
    bounds [2, 2048] and [1000, 100000]."""
    t_ins = min(max(int(round(quadratic(PAPER_T_INSERTION, n))), 2), 2048)
    t_np = min(max(int(round(quadratic(PAPER_T_NUMPY, n))), 1000), 100000)
    return t_ins, t_np


KEY_BYTES = {"int32": 4, "uint32": 4, "float32": 4, "int64": 8, "float64": 8}
DTYPE_CODES = {"int32": 1, "int64": 2, "uint32": 3, "float32": 4, "float64": 5}


def effective_tile(es, dtype_name: str, n: int, params) -> int:
    """Keys per radix tile a keys-only sort of n keys with `params` uses (0 if it takes another routine)."""
    info = es.plan(es.OP_SORT, DTYPE_CODES[dtype_name], n, 0, params)
    return int(info["tile_keys"]) if info["path_name"] == "radix" else 0


def fit_tile_formula(es, table: dict, key_bytes: int) -> Tuple[float, float, float]:
    """The Eq. 1 / Eq. 2 form refit on the GPU table: least-squares quadratic in x = log10(n) of log2(keys per
    radix tile) over the GA's picks for uniform keys of this width (every size class whose pick is the
    radix routine, hand-coded shapes resolved for the digit width and n the pick was made at)."""
    xs, ys = [], []
    for e in table.get("entries", []):
        if e.get("dist") != "uniform" or KEY_BYTES.get(e.get("dtype")) != key_bytes:
            continue
        d = dict(e["params"])
        d["shape"] = tuple(d.get("shape", (0, 0)))
        tile = effective_tile(es, e["dtype"], int(e["n"]), to_params(es, d))
        if tile:
            xs.append(math.log10(e["n"]))
            ys.append(math.log2(tile))
    a, b, c = np.polyfit(np.array(xs), np.array(ys), 2)
    return float(a), float(b), float(c)


# Coefficients of that fit on the packaged table (tests refit them from the
# table): log2(keys per tile) = a x^2 + b x + c, x = log10(n).
GPU_TILE_FORMULA = {4: (-0.0990, 1.9519, 4.9459), 8: (-0.3618, 5.2535, -5.7880)}

# Largest tile the radix pass compiles for keys only at 8-bit digits.
_MAX_TILE = {4: 768 * 24, 8: 768 * 12}


def closed_form_params(es, dtype_name: str, n: int):
    """Library params from the GPU closed form: the compiled tile shape (at 8-bit digits, keys only) whose
    key count is nearest, on a log scale, to 2^(a x^2 + b x + c), at most the largest default tile."""
    kb = KEY_BYTES[dtype_name]
    want = min(2.0 ** quadratic(GPU_TILE_FORMULA[kb], n), _MAX_TILE[kb])
    best, best_d = None, None
    for shape in RADIX_SHAPES[1:]:
        p = to_params(es, {"algo": 4, "digit_bits": 8, "shape": shape})
        try:
            es.plan(es.OP_SORT, DTYPE_CODES[dtype_name], max(n, 2), 0, p)
        except es.EvosortError:
            continue
        d = abs(math.log2(shape[0] * shape[1]) - math.log2(want))
        if best is None or d < best_d - 1e-9 or (abs(d - best_d) <= 1e-9 and shape[0] > best[0]):
            best, best_d = shape, d
    return to_params(es, {"algo": 4, "digit_bits": 8, "shape": best})


# A table entry becomes a row of the compiled table only where the GA's
# re-timed pick beat the re-timed default by this much: smaller gains moved
# between tuning runs by as much as their size (the mergesort for float64 at
# 1e5 keys: 4.5, 2.6, 1.1 and 2.0 % in four runs) and were losses at the ends
# of the row's range (10 % at 1.41e5 keys).
AUTO_MIN_GAIN = 0.05


def _cut(num: int, den: int = 1) -> int:
    """Smallest integer m >= 0 with den * m^2 >= num (an exact ceil(sqrt(num / den)))."""
    m = math.isqrt(num // den)
    while den * m * m < num:
        m += 1
    return m


def auto_table_rows(table: dict):
    """Rows of the table the library compiles in for EVOSORT_ALGO_AUTO: (key type, size class n, lo, hi, A_code),
    one per (key type, size class) whose uniform-key pick is the mergesort and beat the default radix sort by
    AUTO_MIN_GAIN (every entry of that key type and size class, if the table holds several, with the same pick).

    A row applies to keys-only sorts of lo <= n < hi keys, where lo and hi are the geometric means of its size
    class and the neighbouring size classes the table tuned for that key type (half a decade beyond the smallest
    and the largest).  The GA's radix tile picks give no row: timed at the ends of such ranges they lost up to
    9 % to the hand-coded tiles (their gain at the size class itself comes from where that particular n falls
    against the number of workgroups the GPU holds at once, which moves with n), while the routine picks held
    over their whole ranges."""
    picks, classes = {}, {}
    for e in table.get("entries", []):
        if e.get("dist") != "uniform" or e["dtype"] not in KEY_BYTES:
            continue
        dt, n = e["dtype"], int(e["n"])
        classes.setdefault(dt, set()).add(n)
        gain = 1.0 - e["ms"] / e["default_ms"] if e.get("default_ms") else 0.0
        merge = int(e["params"]["algo"]) == 3
        picks.setdefault((dt, n), []).append(3 if merge and gain >= AUTO_MIN_GAIN else None)
    rows = []
    for (dt, n), ps in sorted(picks.items(), key=lambda kv: (DTYPE_CODES[kv[0][0]], kv[0][1])):
        if not (ps and all(p is not None and p == ps[0] for p in ps)):
            continue
        cs = sorted(classes[dt])
        i = cs.index(n)
        lo = _cut(cs[i - 1] * n) if i > 0 else _cut(n * n, 10)
        hi = _cut(n * cs[i + 1]) if i + 1 < len(cs) else _cut(10 * n * n)
        rows.append((dt, n, lo, hi, ps[0]))
    return rows


def emit_header(table: dict) -> str:
    """C++ header with auto_table_rows(table), the table the library compiles in."""
    lines = [
        "// Size classes where the GA tuner picked the mergesort over the radix sort",
        "// for EVOSORT_ALGO_AUTO keys-only sorts (Sec. 4.2, Algorithm 2, run on an",
        "// MI355X): key type (EVOSORT_* dtype code), size class (keys), the lengths",
        "// lo <= n < hi the row applies to (geometric means with the neighbouring",
        "// tuned size classes), A_code.  Written by `python -m",
        "// paper_2505_18681_amd.tuner --emit-header` from the packaged table",
        "// tuned/mi355x.json; do not edit.",
        "#pragma once",
        "",
        "#include <stdint.h>",
        "",
        "namespace evosort {",
        "",
        "struct TunedRow {",
        "    int dtype;",
        "    int64_t n;",
        "    int64_t lo;",
        "    int64_t hi;",
        "    int algo;",
        "};",
        "",
        "constexpr TunedRow kTunedRows[] = {",
    ]
    rows = auto_table_rows(table)
    for dt, n, lo, hi, algo in rows:
        lines.append(f"    {{{DTYPE_CODES[dt]}, {n}, {lo}, {hi}, {algo}}},  // {dt}")
    if not rows:
        lines.append("    {0, 0, 0, 0, 0},")
    lines += ["};", f"constexpr int kTunedRowCount = {len(rows)};", "", "}  // namespace evosort", ""]
    return "\n".join(lines)


HEADER_PATH = __import__("os").path.join(__import__("os").path.dirname(__import__("os").path.abspath(__file__)),
                                         "csrc", "tuned_table.hpp")


def main(argv=None):
    """Tune the sort per key type, size class and distribution (and optionally a batch) on the current GPU and
    write a JSON table."""
    import sys as _sys

    args_in = list(_sys.argv[1:] if argv is None else argv)
    if args_in[:1] == ["--emit-header"]:
        with open(HEADER_PATH, "w") as f:
            f.write(emit_header(packaged_table()))
        print(HEADER_PATH)
        return
    import argparse
    import os
    import sys

    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--dtypes", default="int32", help="comma-separated key types")
    ap.add_argument("--n", default="1e6,1e7,1e8", help="comma-separated sample sizes (size classes)")
    ap.add_argument("--dists", default="uniform", help="comma-separated distributions, or 'all'")
    ap.add_argument("--extra", default="", help="extra dtype:n:dist entries, comma-separated")
    ap.add_argument("--batched-nseg", type=int, default=0, help="also tune the batched sort on this many arrays")
    ap.add_argument("--pop", type=int, default=POP_SIZE)
    ap.add_argument("--generations", type=int, default=GENERATIONS)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--seed", type=int, default=42)
    ap.add_argument("--out", required=True)
    args = ap.parse_args(argv)

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    if root not in sys.path:
        sys.path.insert(0, root)
    import torch

    import paper_2505_18681_amd as es
    import workloads

    dists = list(workloads.DISTRIBUTIONS) if args.dists == "all" else args.dists.split(",")
    jobs = [(dt, int(float(x)), dist) for dt in args.dtypes.split(",") for x in args.n.split(",") for dist in dists]
    for item in filter(None, args.extra.split(",")):
        dt, x, dist = item.split(":")
        jobs.append((dt, int(float(x)), dist))
    table = {"device": torch.cuda.get_device_name(0),
             "ga": {"pop": args.pop, "generations": args.generations, "reps": args.reps, "seed": args.seed},
             "entries": []}
    for dt, n, dist in jobs:
        host = workloads.make(dist, np.dtype(dt), n, args.seed)
        keys = torch.from_numpy(host.view(np.int32) if dt == "uint32" else host).cuda()
        if dt == "uint32":
            keys = keys.view(torch.uint32)
        e = tune_sort(es, keys, seed=args.seed, pop_size=args.pop, generations=args.generations, reps=args.reps)
        e.update({"dtype": dt, "dist": dist})
        table["entries"].append(e)
        print(json.dumps({k: e[k] for k in ("dtype", "dist", "n", "params", "ms", "default_ms", "evaluations")}),
              flush=True)
        del keys, host
        torch.cuda.empty_cache()
    if args.batched_nseg:
        sizes = workloads.segment_sizes(args.batched_nseg, args.seed)
        offs = workloads.segment_offsets(sizes)
        host = workloads.uniform(np.uint32, int(offs[-1]), args.seed)
        keys = torch.from_numpy(host.view(np.int32)).cuda().view(torch.uint32)
        del host
        e = tune_segmented(es, keys, torch.from_numpy(offs).cuda(), seed=args.seed, pop_size=args.pop,
                           generations=args.generations, reps=args.reps)
        e.update({"dtype": "uint32", "dist": "lognormal_batch"})
        table["batched"] = e
        print(json.dumps({k: e[k] for k in ("dtype", "n", "nseg", "params", "ms", "default_ms")}), flush=True)
    save_table(table, args.out)


if __name__ == "__main__":
    main()
