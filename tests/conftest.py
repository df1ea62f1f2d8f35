import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


@pytest.fixture(scope="session")
def world_c1():
    from paper_2107_01715_amd import workload as W
    from oracle import qnet as Q, search as S
    ep = W.env_params(1001)
    return S.World(ep.delta, ep.vel, Q.prepare(W.qnet_weights(7)))
