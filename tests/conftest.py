import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C ABI on the device)")
    config.addinivalue_line("markers", "slow: longer CPU test")


def _ensure_built():
    """Build the HIP library once if nothing is built (tests never rebuild an existing one)."""
    pkg = os.path.join(ROOT, "paper_2607_16946_amd")
    if not (os.path.exists(os.path.join(pkg, "libpts.so")) and os.path.exists(os.path.join(pkg, "libpts_probe.so"))):
        from paper_2607_16946_amd import build
        build.build()


_ensure_built()
