"""Shared test configuration.

Markers: ``gpu`` marks tests that need an MI355X (run with ``-m gpu``); every
other test runs on the CPU.  The CPU oracle is loaded through ``oracle`` and
built on first use if no library is present.
"""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an AMD Instinct MI355X (gfx950)")
    config.addinivalue_line("markers", "slow: long-running oracle physics pin")
