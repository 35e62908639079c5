import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the C-ABI library)")
    config.addinivalue_line("markers", "slow: CPU test that runs the oracle for tens of seconds")


@pytest.fixture(scope="session")
def paper():
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="session", autouse=True)
def _oracle_built():
    from oracle.build import build_oracle
    build_oracle(force=False)
