"""The CPU oracle against values and properties fixed by the paper and by
mathematics (see tests/oracle_pins.py for what each pin checks)."""
import pytest

import oracle
from oracle_pins import ALL_PINS


@pytest.mark.parametrize("pin", ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    pin(oracle.default())
