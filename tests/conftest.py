import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


def pytest_sessionstart(session):
    """Refuse to test a stale native library: every source under csrc/ must be older
    than the built libldpcx.so (run __graft_entry__.build() after editing them)."""
    lib = os.path.join(ROOT, "paper_2508_03567_amd", "libldpcx.so")
    src = os.path.join(ROOT, "paper_2508_03567_amd", "csrc")
    if not os.path.exists(lib):
        return
    built = os.path.getmtime(lib)
    newer = [f for f in os.listdir(src) if os.path.getmtime(os.path.join(src, f)) > built + 5.0]
    if newer:
        raise RuntimeError(f"libldpcx.so is older than {sorted(newer)}: rebuild before testing")
