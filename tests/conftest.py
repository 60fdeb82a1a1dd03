import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_sessionfinish(session, exitstatus):
    """Write what the GPU parity comparisons saw (mismatch counts, worst
    cumulative-weight error, hardware-log error) to a JSON report."""
    parity = sys.modules.get("parity")
    if parity is None or not (parity.REPORT["mismatches"] or parity.REPORT["cumw"]):
        return
    import json
    path = os.environ.get("RS_PARITY_REPORT",
                          os.path.join(ROOT, "results", "parity_report.json"))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"summary": parity.summary(), "exitstatus": int(exitstatus),
                   "records": parity.REPORT}, f, indent=1)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: exhaustive or statistical check taking several seconds")
