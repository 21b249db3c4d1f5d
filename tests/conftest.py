import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: longer CPU test")


@pytest.hookimpl(hookwrapper=True, trylast=True)
def pytest_runtest_call(item):
    """GPU tests print the case they run and their progress straight to the terminal, so a
    long full-size case keeps writing while it runs and a failure is named by its last line."""
    if item.get_closest_marker("gpu") is None:
        yield
        return
    capman = item.config.pluginmanager.getplugin("capturemanager")
    with capman.global_and_fixture_disabled():
        yield
