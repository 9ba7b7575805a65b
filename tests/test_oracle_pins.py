"""The FP64 oracle against its pins (definitions, closed forms, invariants)."""
import pytest

import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(ref, pin):
    pin(ref)
