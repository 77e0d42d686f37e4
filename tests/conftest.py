import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) to run")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    """Write the parity counts the GPU tests recorded (exclusions, largest
    differences and tolerances) as JSON: reports/parity_report.json at the
    repository root unless PV_PARITY_REPORT names another file."""
    from tests import harness
    if not harness.REPORT:
        return
    import json
    path = os.environ.get("PV_PARITY_REPORT", os.path.join(ROOT, "reports", "parity_report.json"))
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump({"exitstatus": int(exitstatus), "comparisons": harness.REPORT}, f, indent=1, sort_keys=True)
