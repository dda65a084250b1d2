import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")


@pytest.fixture(scope="session")
def orc():
    import oracle

    oracle.build(force=False)
    return oracle


@pytest.fixture(scope="session")
def qlib():
    """The HIP library (built in-tree if it is not there yet)."""
    from paper_2601_19034_amd import binding

    if not os.path.exists(binding.LIB_PATH):
        from paper_2601_19034_amd import build

        build.build()
    return binding.load()
