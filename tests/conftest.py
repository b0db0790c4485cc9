import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP library through its C ABI)")
    config.addinivalue_line("markers", "slow: longer CPU test")
    config.addinivalue_line("markers", "mutation: plants one mistake in a scratch copy of the oracle (CPU, opt-in)")


def pytest_addoption(parser):
    parser.addoption("--mutations", action="store_true", default=False,
                     help="run the oracle mutation check (each case plants a mistake in a scratch copy of the "
                          "oracle and expects the CPU pins to fail)")


def pytest_collection_modifyitems(config, items):
    if config.getoption("--mutations"):
        return
    import pytest
    skip = pytest.mark.skip(reason="oracle mutation check: run with --mutations")
    for item in items:
        if "mutation" in item.keywords:
            item.add_marker(skip)
