"""The full-monomer-equation oracle against facts outside itself (CPU only)."""
import pytest

from oracle import mcpt_lccd
from . import pins_lccd


@pytest.mark.parametrize("pin", pins_lccd.ALL_LCCD_PINS, ids=lambda f: f.__name__)
def test_lccd_pin(pin):
    ok, detail = pin(mcpt_lccd)
    assert ok, detail
