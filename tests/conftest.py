import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI on the device)")
    config.addinivalue_line("markers", "slow: large inputs (minutes on the CPU)")


def _ensure_built():
    """Build the CPU-side libraries once if they are missing (the GPU library
    is built by __graft_entry__.build(); tests never compile HIP code)."""
    import __graft_entry__ as ge
    for path, fn in ((ge.GEN_SO, ge.build_generator), (ge.ORACLE_SO, ge.build_oracle)):
        if not os.path.exists(path):
            fn()


_ensure_built()
