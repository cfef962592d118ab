"""The CPU oracle against facts fixed outside it (see oracle_pins.py)."""
import pytest

import oracle_pins
from oracle.oracle import default


@pytest.fixture(scope="module")
def O():
    return default()


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(O, pin):
    try:
        pin(O)
    except oracle_pins.AtenUnavailable as e:
        pytest.skip(f"ATen Philox header unavailable: {e}")
