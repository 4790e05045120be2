import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU-only oracle runs")


@pytest.fixture(scope="session")
def spec():
    import synthetic
    return synthetic.ani2x_like_spec()


@pytest.fixture(scope="session")
def spec_bias():
    """Same model with non-zero biases and self energies, so bias paths are exercised."""
    import synthetic
    return synthetic.ani2x_like_spec(weight_seed=777, bias_scale=0.1,
                                     self_energy=[-0.5, -38.0, -54.6, -75.0, -99.7, -398.1, -460.1])
