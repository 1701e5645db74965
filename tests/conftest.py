import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

GOLDEN = ROOT / "tests" / "golden"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: large inputs (still CPU-feasible)")


def read_golden(name):
    """Parse a `key v1 v2 ...` text fixture ('#' starts a comment)."""
    out = {}
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        key, *vals = line.split()
        out[key] = vals
    return out


@pytest.fixture(scope="session")
def golden():
    return read_golden
