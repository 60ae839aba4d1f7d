import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")
    config.addinivalue_line("markers", "slow: large CPU case")


@pytest.fixture(scope="session")
def hex_sphere_wl():
    from synth import workloads
    return workloads.hex_sphere()


@pytest.fixture(scope="session")
def small_voronoi_wl():
    from synth import workloads
    return workloads.voronoi_bubble(n=12, seed=7, r=0.3)
