import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


@pytest.fixture(scope="session")
def orc():
    import oracle
    return oracle.Oracle()


@pytest.fixture(scope="session")
def ev_plain():
    from paper_1911_09340_amd import synth
    return synth.event_plain(0)


@pytest.fixture(scope="session")
def ev_plain_exact():
    from paper_1911_09340_amd import synth
    return synth.event_plain(0, sigma=0.0)


@pytest.fixture(scope="session")
def ev_signal():
    from paper_1911_09340_amd import synth
    return synth.event_signal(0)
