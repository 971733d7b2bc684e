import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: oracle runs that take more than a few seconds")


@pytest.fixture
def record_error(request):
    """record_error(what, value, bar): note an achieved error beside the bar it is
    held to.  With PSMS_ERROR_LOG set, each record is appended to that file as one
    JSON line (test id, quantity, value, bar); otherwise nothing is written."""
    import json

    path = os.environ.get("PSMS_ERROR_LOG")

    def rec(what, value, bar=None):
        if path:
            with open(path, "a") as f:
                f.write(json.dumps({"test": request.node.nodeid, "what": str(what), "value": float(value),
                                    "bar": None if bar is None else float(bar)}) + "\n")
        return value

    return rec
