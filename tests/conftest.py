import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_collection_modifyitems(session, config, items):
    """When GPU tests are selected, start the oracle worker pool now: after
    collection, before any test initialises the GPU (the workers are forked)."""
    if not any(item.get_closest_marker("gpu") for item in items):
        return
    torch = sys.modules.get("torch")
    if torch is not None and torch.cuda.is_initialized():
        return
    from tests import oracle_pool
    oracle_pool.start()


def pytest_sessionfinish(session, exitstatus):
    mod = sys.modules.get("tests.oracle_pool")
    if mod is not None:
        mod.stop()
