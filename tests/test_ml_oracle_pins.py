"""The application oracles (SPADE densities, L1 assign, naive Bayes, GDA)
against their pins (CPU only)."""
import pytest

import ml_pins
from oracle import ml


@pytest.fixture(scope="module")
def lib():
    return ml.build()


@pytest.mark.parametrize("pin", ml_pins.ALL_ML_PINS, ids=lambda f: f.__name__)
def test_pin(pin, lib):
    pin(lib)
