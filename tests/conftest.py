import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long CPU-only check, run with LBM_SLOW=1")


def pytest_collection_modifyitems(config, items):
    import pytest
    if os.environ.get("LBM_SLOW") == "1":
        return
    skip = pytest.mark.skip(reason="slow CPU check; set LBM_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)
