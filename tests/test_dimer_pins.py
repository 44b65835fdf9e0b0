"""The dimer-internal oracle against facts outside itself (CPU only)."""
import pytest

from oracle import mcpt_dimer
from . import pins_dimer


@pytest.mark.parametrize("pin", pins_dimer.ALL_PINS, ids=lambda f: f.__name__)
def test_dimer_pin(pin):
    ok, detail = pin(mcpt_dimer)
    assert ok, detail
