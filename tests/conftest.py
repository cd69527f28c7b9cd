import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(autouse=True, scope="session")
def _torch_threads():
    import torch
    torch.set_num_threads(min(8, os.cpu_count() or 1))
    yield


@pytest.fixture(scope="session")
def pgo():
    """The product binding with libpgo.so built (built here only if missing
    or older than its sources)."""
    from paper_2601_15684_amd import build as B
    if B.is_stale():
        B.build()
    import paper_2601_15684_amd as P
    P.lib()
    return P


def pytest_terminal_summary(terminalreporter):
    """The raw parity errors of every GPU comparison and their bounds
    (tests/tolerance.py); also written to $PGO_PARITY_REPORT when set."""
    import sys as _sys
    T = _sys.modules.get("tests.tolerance")
    if T is None or not T.REPORT:
        return
    text = T.format_report()
    terminalreporter.write_line(text)
    path = os.environ.get("PGO_PARITY_REPORT")
    if path:
        with open(path, "w") as f:
            f.write(text + "\n")
