import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    oracle.load()
    return oracle


@pytest.fixture(scope="session")
def tiny():
    import synth
    return synth.make_workload("tiny")


@pytest.fixture(scope="session")
def tiny_grids(orc, tiny):
    return orc.workload_grids(tiny)


@pytest.fixture(scope="session")
def paper():
    import synth
    return synth.make_workload("paper")


@pytest.fixture(scope="session")
def paper_grids(orc, paper):
    return orc.workload_grids(paper)
