import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# Mutation tests re-run the oracle pins against a deliberately broken copy of
# the oracle in a temporary directory: a mutated C library
# (EVOSORT_TEST_ORACLE_MUTANT, the path of the .so) or a mutated copy of the
# whole package (EVOSORT_TEST_ORACLE_PKG, the directory holding it).  Nothing
# outside the tests sets either.
_MUTANT_PKG = os.environ.get("EVOSORT_TEST_ORACLE_PKG")
if _MUTANT_PKG:
    sys.path.insert(0, _MUTANT_PKG)
    import oracle as _oracle_pkg

    assert os.path.dirname(os.path.dirname(os.path.abspath(_oracle_pkg.__file__))) == os.path.abspath(_MUTANT_PKG)
_MUTANT = os.environ.get("EVOSORT_TEST_ORACLE_MUTANT")
if _MUTANT:
    import oracle as _oracle

    _oracle._LIB_PATH = _MUTANT
    _oracle._lib = None


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "full_size: GPU parity at full benchmark sizes (minutes, >100 GB of HBM)")


def golden_path(name: str) -> str:
    return os.path.join(ROOT, "tests", "golden", name)


def read_golden(name: str):
    rows = []
    with open(golden_path(name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture
def golden():
    return read_golden
