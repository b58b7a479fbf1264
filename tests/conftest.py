import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
HERE = os.path.dirname(os.path.abspath(__file__))
if HERE not in sys.path:
    sys.path.insert(0, HERE)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


def pytest_collection_finish(session):
    """Start the sharded oracle run of the full MR-like workload when a test that
    needs it was selected and the machine has a GPU.  The check reads the device
    node only, so the pool forks from a process without HIP state."""
    import oracle_pool

    if not any(item.name in oracle_pool.USERS for item in session.items):
        return
    if not os.path.exists("/dev/kfd"):
        return
    oracle_pool.start()


def pytest_sessionfinish(session, exitstatus):
    import oracle_pool

    oracle_pool.stop()
