"""The singles oracle against facts outside itself (CPU only)."""
import pytest

from oracle import mcpt_singles
from . import pins_singles


@pytest.mark.parametrize("pin", pins_singles.ALL_SINGLES_PINS, ids=lambda f: f.__name__)
def test_singles_pin(pin):
    ok, detail = pin(mcpt_singles)
    assert ok, detail
