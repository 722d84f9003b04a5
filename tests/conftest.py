import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: larger CPU cases")


def pytest_sessionfinish(session, exitstatus):
    """With the check build loaded (BC_MI355X_CHECK_EXEC=1), report the
    cross-lane helper calls made with part of a wave inactive over the whole
    session, and fail the session if there were any."""
    if os.environ.get("BC_MI355X_CHECK_EXEC", "") != "1":
        return
    from paper_2401_02472_amd import _capi
    if _capi._lib is None:
        return
    count = int(_capi._lib.bc_debug_exec_partial())
    print(f"\ncross-lane helper calls with part of a wave inactive: {count}", flush=True)
    if count != 0:
        session.exitstatus = 1
