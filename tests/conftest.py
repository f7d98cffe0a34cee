import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def _gpu_visible():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.fixture(scope="session")
def gpu_required():
    if not _gpu_visible():
        pytest.skip("no GPU visible")
    from paper_1702_06359_amd import abi
    if not os.path.exists(abi.LIB_PATH):
        pytest.fail("libmkf.so is not built (run __graft_entry__.build())")
    return True


def report(name, payload):
    """Print a measurement (flushed) and, when MKF_REPORT_DIR is set, keep it as JSON."""
    import json
    line = json.dumps({"case": name, **payload}, default=float)
    print(line, flush=True)
    d = os.environ.get("MKF_REPORT_DIR")
    if d:
        os.makedirs(d, exist_ok=True)
        with open(os.path.join(d, "reports.jsonl"), "a") as f:
            f.write(line + "\n")
