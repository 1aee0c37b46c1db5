import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a real MI355X (HIP device)")
    config.addinivalue_line("markers", "slow: large CPU-side workloads")


@pytest.fixture(scope="session")
def tiny_mesh():
    from synth import config_mesh
    return config_mesh("tiny")


@pytest.fixture(scope="session")
def tiny_oracle(tiny_mesh):
    import oracle
    return oracle.OracleMesh.from_kuhn(tiny_mesh)
