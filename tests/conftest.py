import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


# Mutation tests re-run the oracle pins against a deliberately broken copy of
# the oracle built in a temporary directory; they point the oracle package at
# that copy through this variable.  Nothing outside the tests sets it.
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
