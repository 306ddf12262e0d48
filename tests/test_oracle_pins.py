"""The CPU oracle against facts that the paper and mathematics fix (see
``pins.py``).  Runs on the CPU only."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin, oracle_lib):
    pin(oracle_lib)
