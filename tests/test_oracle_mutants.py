"""Plant plausible mistakes in a copy of the oracle and check that the pins catch each one.

Every mutant is a one-token change of ``oracle/evosort_oracle.c`` (a flipped
tie rule, a wrong mask, a dropped complement, a shifted digit, an off-by-one in
a count), compiled into a temporary directory, or of the dispatch rule in
``oracle/__init__.py`` (each clause of the adaptive partition sort), copied
with the rest of the package into a temporary directory.  The pin suite is
re-run against it in a child process; the test passes only if that run fails.
The real oracle is never modified.  Mutants are chosen so that none can write
out of bounds.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "evosort_oracle.c")

MUTANTS = {
    "mergesort tie takes the right run": (
        "descending ? (r[b].u > r[a].u) : (r[b].u < r[a].u);",
        "descending ? (r[b].u > r[a].u) : (r[b].u <= r[a].u);"),
    "descending mergesort tie takes the right run": (
        "descending ? (r[b].u > r[a].u) : (r[b].u < r[a].u);",
        "descending ? (r[b].u >= r[a].u) : (r[b].u < r[a].u);"),
    "descending direction ignored": (
        "mergesort_records(r, tmp, 0, n, descending ? 1 : 0);", "mergesort_records(r, tmp, 0, n, 0);"),
    "int32 offset off by one": ("(int64_t)v + 2147483648LL", "(int64_t)v + 2147483647LL"),
    "int64 offset wrong bit": ("return (uint64_t)v + (UINT64_C(1) << 63);", "return (uint64_t)v + (UINT64_C(1) << 62);"),
    "float32 negative not complemented": ("return (uint64_t)(uint32_t)~b;", "return (uint64_t)b;"),
    "float64 positive sign bit not set": ("return b | (UINT64_C(1) << 63);", "return b;"),
    "counting pass reads the wrong digit": (
        "        next[(u >> shift) & (bins - 1)] += 1;", "        next[(u >> (shift + 1)) & (bins - 1)] += 1;"),
    "histogram drops the pass index": ("hist[(uint64_t)p * bins + d] += 1;", "hist[d] += 0 * p + 1;"),
    "insertion sort unstable": ("while (j >= lo && r[j].u > x.u)", "while (j >= lo && r[j].u >= x.u)"),
    "merge round tie takes the right run": (
        "            if (r[b].u < r[a].u)\n                perm_out[k++] = r[b++].idx;",
        "            if (r[b].u <= r[a].u)\n                perm_out[k++] = r[b++].idx;"),
    "rank counts the element itself": ("(uk == ui && k < i)", "(uk == ui && k <= i)"),
    "unsorted check compares the wrong way": (
        "order_key(kind, base, j) > order_key(kind, base, j + 1)",
        "order_key(kind, base, j) < order_key(kind, base, j + 1)"),
}


# One-token changes of the dispatch rule (Sec. 4.3, Algorithm 6, with the
# library's readings), one per clause.
PY_MUTANTS = {
    "small branch ignores the one-workgroup capacity": (
        "if n < t_fallback and n <= small_capacity:", "if n < t_fallback:"),
    "capacity compared strictly": (
        "if n < t_fallback and n <= small_capacity:", "if n < t_fallback and n < small_capacity:"),
    "fallback threshold not strict": (
        "if n < t_fallback and n <= small_capacity:", "if n <= t_fallback and n <= small_capacity:"),
    "A_code 0 is not automatic": (
        "if a_code in (0, A_RADIX) and (integer_keys or radix_for_floats):",
        "if a_code == A_RADIX and (integer_keys or radix_for_floats):"),
    "float keys never take the radix branch": (
        "if a_code in (0, A_RADIX) and (integer_keys or radix_for_floats):",
        "if a_code in (0, A_RADIX) and integer_keys:"),
    "float keys always take the radix branch": (
        "if a_code in (0, A_RADIX) and (integer_keys or radix_for_floats):",
        "if a_code in (0, A_RADIX):"),
    "A_code 3 takes the radix branch": (
        "if a_code in (0, A_RADIX) and (integer_keys or radix_for_floats):",
        "if a_code in (0, 3, A_RADIX) and (integer_keys or radix_for_floats):"),
}


def _run_pins(env):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_pins_catch_planted_dispatch_mistake(name, tmp_path):
    before, after = PY_MUTANTS[name]
    pkg = os.path.join(ROOT, "oracle")
    src = open(os.path.join(pkg, "__init__.py")).read()
    assert src.count(before) == 1, f"mutation site not unique or missing: {name}"
    dst = tmp_path / "oracle"
    dst.mkdir()
    for f in ("evosort_oracle.c", "build.py", "liboracle.so"):
        if os.path.exists(os.path.join(pkg, f)):
            shutil.copy(os.path.join(pkg, f), dst / f)
    (dst / "__init__.py").write_text(src.replace(before, after))
    env = dict(os.environ, EVOSORT_TEST_ORACLE_PKG=str(tmp_path))
    r = _run_pins(env)
    assert r.returncode != 0, f"pins did not catch mutant {name!r}:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "Error" in r.stdout


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_planted_mistake(name, tmp_path):
    before, after = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(before) == 1, f"mutation site not unique or missing: {name}"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(before, after))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", str(mutant_c), "-o", str(lib)], check=True)
    env = dict(os.environ, EVOSORT_TEST_ORACLE_MUTANT=str(lib))
    r = _run_pins(env)
    assert r.returncode != 0, f"pins did not catch mutant {name!r}:\n{r.stdout[-2000:]}"
    assert "failed" in r.stdout or "Error" in r.stdout
