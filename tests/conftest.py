import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def c1():
    from paper_2605_13987_amd import workloads
    return workloads.config_c1()


@pytest.fixture(scope="session")
def c1_oracle(c1):
    import oracle
    return oracle.weighting_field(c1["cell"], c1["columns"], c1["spectrum"])
