"""The CPU oracle against closed forms, exact arithmetic, LAPACK and the
identities of Section 3 (see oracle_pins.py for what each pin fixes)."""
import pytest

import oracle
from oracle_pins import PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_pin(pin):
    pin(oracle.default())
