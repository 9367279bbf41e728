"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws numbers: it holds none of the sort's arithmetic, and it
imports neither the GPU library nor the oracle.  Every generator is a pure
function of (size, seed) built on numpy's PCG64 generator.

Distributions (the paper's own inputs are synthetic integer arrays drawn with a
fixed seed, 42 by default, Sec. 7.5 and the data availability statement):

* ``uniform``        -- i.i.d. uniform over the full bit range of the dtype
                        (floats: uniform bit patterns, NaN patterns redrawn);
* ``gaussian``       -- round(N(0, sd)) clipped to the dtype's range (int);
* ``sorted``         -- non-decreasing: a running sum of random gaps, so no
                        sort is needed to make it;
* ``reverse``        -- the same sequence reversed;
* ``nearly_sorted``  -- ``sorted`` with a fraction of random position swaps;
* ``distinct16``     -- 16 distinct values drawn once, then chosen uniformly;
* ``zipf``           -- rank r in 1..ranks with P(r) proportional to r**-s;
* ``all_equal``      -- every key 42;
* ``float_mix``      -- N(0, 1) with a fraction replaced by values drawn from
                        {-inf, +inf, -0.0, +0.0} (no NaN).

The paper's own nine int32 distributions (its experimental setup lists them,
all mapped to [-1e9, 1e9]; ``paper_*`` names, :data:`PAPER_DISTRIBUTIONS`):
uniform, normal (sd 1e8), exponential (scale 1e9), power law (a = 0.5), beta
(2, 5), sparse (90 % zeros), clustered (10 centres, sd 1e8), nearly sorted (a
linear ramp with 10 % of positions replaced at random) and duplicates (10 %
distinct values).  They are drawn here with numpy's Generator API, so the
values differ from the paper's legacy-seeded arrays; the shapes follow its
recipe.

Batches of arrays: :func:`segment_sizes` draws log-normal array sizes
(round(exp(N(ln median, sigma))), clipped), :func:`segment_offsets` turns sizes
into the nseg + 1 offsets of one buffer.
"""
from __future__ import annotations

import numpy as np

DEFAULT_SEED = 42

DISTRIBUTIONS = (
    "uniform",
    "gaussian",
    "sorted",
    "reverse",
    "nearly_sorted",
    "distinct16",
    "zipf",
    "all_equal",
)

PAPER_DISTRIBUTIONS = (
    "paper_uniform",
    "paper_normal",
    "paper_exponential",
    "paper_power",
    "paper_beta",
    "paper_sparse",
    "paper_clustered",
    "paper_nearly_sorted",
    "paper_duplicates",
)

_LIM = 1_000_000_000  # the paper maps every distribution to [-1e9, 1e9]


def paper_distribution(name: str, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """One of the paper's nine int32 distributions (see the module docstring)."""
    g = rng(seed)
    if name == "paper_uniform":
        return g.integers(-_LIM, _LIM, size=n, dtype=np.int64).astype(np.int32)
    if name == "paper_normal":
        return np.clip(g.normal(0.0, 1e8, size=n), -_LIM, _LIM).astype(np.int32)
    if name == "paper_exponential":
        return (np.clip(g.exponential(1e9, size=n), 0, 2 * _LIM) - _LIM).astype(np.int32)
    if name == "paper_power":
        return (g.power(0.5, size=n) * 2 * _LIM - _LIM).astype(np.int32)
    if name == "paper_beta":
        return (g.beta(2.0, 5.0, size=n) * 2 * _LIM - _LIM).astype(np.int32)
    if name == "paper_sparse":
        out = np.zeros(n, dtype=np.int32)
        k = n // 10
        pos = g.choice(n, size=k, replace=False)
        out[pos] = g.integers(-_LIM, _LIM, size=k, dtype=np.int64).astype(np.int32)
        return out
    if name == "paper_clustered":
        centres = np.linspace(-_LIM, _LIM, 10)
        c = centres[g.integers(0, 10, size=n)]
        return np.clip(g.normal(c, 1e8), -_LIM, _LIM).astype(np.int32)
    if name == "paper_nearly_sorted":
        out = np.linspace(-_LIM, _LIM, n).astype(np.int32)
        k = n // 10
        pos = g.choice(n, size=k, replace=False)
        out[pos] = g.integers(-_LIM, _LIM, size=k, dtype=np.int64).astype(np.int32)
        return out
    if name == "paper_duplicates":
        uniq = g.integers(-_LIM, _LIM, size=max(1, n // 10), dtype=np.int64).astype(np.int32)
        return uniq[g.integers(0, uniq.size, size=n)]
    raise ValueError(f"unknown distribution {name!r}")


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def _int_bounds(dtype):
    info = np.iinfo(dtype)
    return int(info.min), int(info.max)


def uniform(dtype, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """i.i.d. uniform over every bit pattern of ``dtype`` (NaN patterns excluded for floats)."""
    dtype = np.dtype(dtype)
    g = rng(seed)
    if dtype.kind in "iu":
        lo, hi = _int_bounds(dtype)
        return g.integers(lo, hi, size=n, dtype=dtype, endpoint=True)
    if dtype == np.float32:
        bits = g.integers(0, 2**32 - 1, size=n, dtype=np.uint32, endpoint=True)
        out = bits.view(np.float32)
        bad = np.isnan(out)
        while bad.any():
            bits[bad] = g.integers(0, 2**32 - 1, size=int(bad.sum()), dtype=np.uint32, endpoint=True)
            bad = np.isnan(out)
        return out
    if dtype == np.float64:
        bits = g.integers(0, 2**64 - 1, size=n, dtype=np.uint64, endpoint=True)
        out = bits.view(np.float64)
        bad = np.isnan(out)
        while bad.any():
            bits[bad] = g.integers(0, 2**64 - 1, size=int(bad.sum()), dtype=np.uint64, endpoint=True)
            bad = np.isnan(out)
        return out
    raise TypeError(f"unsupported dtype {dtype}")


def gaussian(dtype, n: int, seed: int = DEFAULT_SEED, sd: float = 1e6) -> np.ndarray:
    dtype = np.dtype(dtype)
    g = rng(seed)
    x = g.normal(0.0, sd, size=n)
    if dtype.kind in "iu":
        lo, hi = _int_bounds(dtype)
        return np.clip(np.rint(x), lo, hi).astype(dtype)
    return x.astype(dtype)


def sorted_run(dtype, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """A non-decreasing integer sequence spanning most of the dtype's range."""
    dtype = np.dtype(dtype)
    if dtype.kind not in "iu":
        raise TypeError("sorted_run is defined for integer dtypes")
    g = rng(seed)
    lo, hi = _int_bounds(dtype)
    if n == 0:
        return np.empty(0, dtype=dtype)
    span = hi - lo
    gap_max = max(1, min(span // max(n, 1), 2**62) * 2)
    gaps = g.integers(0, gap_max, size=n, dtype=np.uint64)
    gaps[0] = 0
    acc = np.cumsum(gaps, dtype=np.uint64)
    if int(acc[-1]) > span:
        acc = (acc.astype(np.float64) * (span / float(acc[-1]))).astype(np.uint64)
    if dtype.itemsize == 8 and dtype.kind == "i":
        return (acc.astype(np.int64) + np.int64(lo)).astype(dtype)
    return (acc.astype(np.int64) + lo).astype(dtype)


def nearly_sorted(dtype, n: int, seed: int = DEFAULT_SEED, frac: float = 0.01) -> np.ndarray:
    a = sorted_run(dtype, n, seed)
    g = rng(seed + 7919)
    swaps = int(frac * n)
    if n >= 2 and swaps:
        i = g.integers(0, n, size=swaps)
        j = g.integers(0, n, size=swaps)
        for s in range(0, swaps, 1 << 20):
            ii, jj = i[s:s + (1 << 20)], j[s:s + (1 << 20)]
            # sequential semantics for repeated positions are not needed: the
            # result is a fixed function of the seed either way
            tmp = a[ii].copy()
            a[ii] = a[jj]
            a[jj] = tmp
    return a


def distinct16(dtype, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    g = rng(seed)
    pool = uniform(dtype, 16, seed + 1)
    return pool[g.integers(0, 16, size=n)]


def zipf(dtype, n: int, seed: int = DEFAULT_SEED, s: float = 1.1, ranks: int = 1_000_000) -> np.ndarray:
    """Ranks 1..ranks with P(r) proportional to r**-s (truncated Zipf), by inverse CDF."""
    g = rng(seed)
    w = np.arange(1, ranks + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    u = g.random(size=n)
    r = np.searchsorted(cdf, u, side="left") + 1
    return np.minimum(r, ranks).astype(dtype)


def all_equal(dtype, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    del seed
    return np.full(n, 42, dtype=dtype)


def float_mix(dtype, n: int, seed: int = DEFAULT_SEED, frac: float = 0.01) -> np.ndarray:
    """N(0, 1) with ``frac`` of the entries replaced by values from {-inf, +inf, -0.0, +0.0}."""
    dtype = np.dtype(dtype)
    g = rng(seed)
    x = g.normal(0.0, 1.0, size=n).astype(dtype)
    k = int(frac * n)
    if k:
        pos = g.choice(n, size=k, replace=False) if n < (1 << 24) else g.integers(0, n, size=k)
        specials = np.array([-np.inf, np.inf, -0.0, 0.0], dtype=dtype)
        x[pos] = specials[g.integers(0, 4, size=k)]
    return x


def float_edges(dtype) -> np.ndarray:
    """The float edge values, each once, in no particular order."""
    dtype = np.dtype(dtype)
    fi = np.finfo(dtype)
    tiny_sub = np.nextafter(dtype.type(0), dtype.type(1))
    vals = [np.inf, -np.inf, fi.max, -fi.max, fi.tiny, -fi.tiny, tiny_sub, -tiny_sub, 0.0, -0.0,
            1.0, -1.0, 1.5, -1.5]
    return np.array(vals, dtype=dtype)


def make(dist: str, dtype, n: int, seed: int = DEFAULT_SEED) -> np.ndarray:
    """Generator by name (see the module docstring)."""
    if dist.startswith("paper_"):
        if np.dtype(dtype) != np.int32:
            raise ValueError("the paper's distributions are int32")
        return paper_distribution(dist, n, seed)
    if dist == "uniform":
        return uniform(dtype, n, seed)
    if dist == "gaussian":
        return gaussian(dtype, n, seed)
    if dist == "sorted":
        return sorted_run(dtype, n, seed)
    if dist == "reverse":
        return sorted_run(dtype, n, seed)[::-1].copy()
    if dist == "nearly_sorted":
        return nearly_sorted(dtype, n, seed)
    if dist == "distinct16":
        return distinct16(dtype, n, seed)
    if dist == "zipf":
        return zipf(dtype, n, seed)
    if dist == "all_equal":
        return all_equal(dtype, n, seed)
    if dist == "float_mix":
        return float_mix(dtype, n, seed)
    raise ValueError(f"unknown distribution {dist!r}")


def segment_sizes(nseg: int, seed: int = DEFAULT_SEED, median: float = 2048.0, sigma: float = 2.0,
                  lo: int = 16, hi: int = 4_000_000) -> np.ndarray:
    """``nseg`` array sizes: round(exp(N(ln median, sigma))) clipped to [lo, hi] (int64).

    ``sigma`` is in natural-log units.
    """
    g = rng(seed)
    sizes = np.rint(np.exp(g.normal(np.log(median), sigma, size=nseg)))
    return np.clip(sizes, lo, hi).astype(np.int64)


def segment_offsets(sizes) -> np.ndarray:
    """Offsets (int64, len(sizes) + 1) of segments of the given sizes laid end to end from 0."""
    sizes = np.asarray(sizes, dtype=np.int64)
    out = np.zeros(sizes.size + 1, dtype=np.int64)
    np.cumsum(sizes, out=out[1:])
    return out
