import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parent.parent
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

GOLDEN = Path(__file__).resolve().parent / "golden"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")


def read_golden(name: str) -> dict:
    """Parse a `name = value` fixture under tests/golden (comments start with #)."""
    out = {}
    for line in (GOLDEN / name).read_text().splitlines():
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = (s.strip() for s in line.split("=", 1))
        out[k] = v
    return out


@pytest.fixture(scope="session")
def O():
    import oracle

    # ORACLE_LIB_PATH lets the mutation test run these pins against a copy of
    # the oracle with a planted mistake.
    alt = os.environ.get("ORACLE_LIB_PATH")
    return oracle.Oracle(oracle.load(Path(alt)) if alt else None)


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library, bound through its C ABI; the test fails if it is absent."""
    import torch

    if not torch.cuda.is_available():
        pytest.fail("GPU test collected on a machine without a GPU")
    from paper_2301_10904_amd import pir

    return pir.load()


def cpu_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))
