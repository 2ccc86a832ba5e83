import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")

import pytest


@pytest.fixture(scope="session")
def ctx():
    import paper_1110_4623_amd as sp
    c = sp.Context(0)
    print(f"\n[gpu] {c.info}", flush=True)
    yield c
    c.close()


def announce(*parts):
    """Print what a GPU step is about to run (flushed before the launch)."""
    print("[gpu-step]", *parts, flush=True)


def pytest_sessionstart(session):
    """Build the HIP library once if it is not there (tests load what is built)."""
    lib = os.path.join(ROOT, "paper_1110_4623_amd", "libsp.so")
    if not os.path.exists(lib):
        sys.path.insert(0, ROOT)
        import __graft_entry__
        __graft_entry__._builder().build()
