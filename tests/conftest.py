import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: CPU test that takes more than a few seconds")


@pytest.fixture(scope="session")
def model_dict():
    with open(os.path.join(ROOT, "paper_2303_08123_amd", "data", "model_default.json")) as fh:
        return json.load(fh)


@pytest.fixture(scope="session")
def params(model_dict):
    from oracle.model import Params
    return Params.from_dict(model_dict)


@pytest.fixture(scope="session")
def golden():
    with open(os.path.join(ROOT, "tests", "golden", "paper_values.json")) as fh:
        return json.load(fh)


@pytest.fixture
def rng():
    return np.random.default_rng(12345)
