import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def small_workload():
    import synthdata
    return synthdata.make_workload("gauss128")


@pytest.fixture(scope="session")
def small_index(small_workload):
    """Oracle fit of the 10,000 x 128 Gaussian workload: IVF 64 lists, K_c = 10."""
    import oracle
    w = small_workload
    return oracle.fit(w["base"], w["calib"], nlist=64, kmeans_iters=25, calib_k=10, calib_nprobe=8,
                      seed=7)
