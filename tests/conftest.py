import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def pytest_sessionstart(session):
    """DFAMIN_TEST_TUNING='{"field": value, ...}' applies a library tuning to the
    whole run (for sweeping the GPU suite over code paths that the default
    tuning leaves to large inputs).  Tests that change the tuning restore
    this one afterwards."""
    import json
    spec = os.environ.get("DFAMIN_TEST_TUNING")
    if not spec:
        return
    from paper_2508_20735_amd import binding as B
    B.set_tuning(**json.loads(spec))
    print(f"tuning for this run: {B.get_tuning()}", flush=True)
