import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP library)")
    config.addinivalue_line("markers", "slow: oracle work of more than a few seconds")


@pytest.fixture(scope="session")
def sphere1():
    """Sphere of radius 0.5 wavelength, icosphere frequency 10: 2000 triangles, 3000 RWGs."""
    import synth
    return synth.icosphere(10, 0.5)


@pytest.fixture(scope="session")
def rwg1(sphere1):
    from oracle import efie
    return efie.RWG(*sphere1)


@pytest.fixture(scope="session")
def dense1(rwg1):
    from oracle import efie
    return efie.dense_z(rwg1)
