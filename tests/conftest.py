import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# parallel test workers (pytest -n) each get one oracle thread rather than all of the host's
if "PYTEST_XDIST_WORKER" in os.environ:
    os.environ["OMP_NUM_THREADS"] = "1"


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: larger CPU cases")


@pytest.fixture(scope="session")
def cfg_c0():
    from paper_2009_00946_amd import synth
    return synth.load_config("c0_tiny")


@pytest.fixture(scope="session")
def cfg_t1():
    from paper_2009_00946_amd import synth
    return synth.load_config("t1_mixed")


@pytest.fixture(scope="session")
def orc_c0(cfg_c0):
    from oracle import Oracle
    return Oracle(cfg_c0)


@pytest.fixture(scope="session")
def orc_t1(cfg_t1):
    from oracle import Oracle
    return Oracle(cfg_t1)
