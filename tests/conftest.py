import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture
def opt(eng):
    """opt(name, value): set a context option of the module's engine for one
    test; every option it touched is restored afterwards."""
    saved = {}

    def set_(name, value):
        if name not in saved:
            saved[name] = eng.get_option(name)
        eng.set_option(name, int(value))

    yield set_
    for k, v in saved.items():
        eng.set_option(k, v)
