"""The oracle against facts outside itself (CPU only)."""
import pytest

from oracle import mcpt_oracle
from . import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS + [pins.pin_divergence_detected],
                         ids=lambda f: f.__name__)
def test_pin(pin):
    ok, detail = pin(mcpt_oracle)
    assert ok, detail
