"""The CPU oracle against what the paper and the mathematics fix."""
import pytest

from tests import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin):
    errs = pin(None)
    assert errs == [], "\n".join(errs[:10])
