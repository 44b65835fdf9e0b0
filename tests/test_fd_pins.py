"""The finite-displacement oracle against facts outside itself (CPU only)."""
import pytest

from oracle import mcpt_fd
from . import pins_fd


@pytest.mark.parametrize("pin", pins_fd.ALL_FD_PINS, ids=lambda f: f.__name__)
def test_fd_pin(pin):
    ok, detail = pin(mcpt_fd)
    assert ok, detail
