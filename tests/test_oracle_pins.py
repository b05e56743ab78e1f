"""The oracle against its pins (closed forms, invariants, brute force,
textbook traversal, HEALPix identities, finite differences)."""

import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(orc, pin):
    pin(orc, orc.load())
