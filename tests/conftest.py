import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def px32():
    from paper_2605_13987_amd import workloads
    return workloads.uniform_pixel_32x32x64()


@pytest.fixture(scope="session")
def px32_oracle(px32):
    import oracle
    return oracle.weighting_field(px32["cell"], px32["columns"], px32["spectrum"])
