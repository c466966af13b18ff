"""Shared test set-up.

Markers: ``gpu`` marks tests that need an MI355X (gfx950) and the built HIP
library; everything else runs on the CPU.  The oracle is built on first use
when no built copy exists.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
for sub in ("", "oracle"):
    path = os.path.join(ROOT, sub)
    if path not in sys.path:
        sys.path.insert(0, path)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X GPU and the built HIP library")


@pytest.fixture(scope="session")
def orc():
    import hsga_oracle
    if not os.path.exists(hsga_oracle.LIB):
        hsga_oracle.build()
    hsga_oracle.load()
    return hsga_oracle
