import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


_GBUFFERS = {}


@pytest.fixture(scope="session")
def workload_gbuffer():
    """(room, G-buffer) of a workload's first frame at full size, built once
    per test session (the 3840x2160 frame with its meshes takes about a
    minute on the host)."""
    def get(name):
        if name not in _GBUFFERS:
            from niv_synth import get_workload, make_workload_gbuffer
            _GBUFFERS[name] = make_workload_gbuffer(get_workload(name))
        return _GBUFFERS[name]
    return get
