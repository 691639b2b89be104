"""The CPU oracle against closed forms, invariants, independent methods and
finite differences (see ``pins.py``)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(orc, pin):
    pin(orc)
