import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long CPU run, opt in with -m slow")


def pytest_collection_modifyitems(config, items):
    import pytest
    if os.environ.get("PMS_RUN_SLOW"):
        return
    skip = pytest.mark.skip(reason="slow CPU run; set PMS_RUN_SLOW=1 to include")
    for item in items:
        if "slow" in item.keywords:
            item.add_marker(skip)
