"""Planted mistakes in the finite-displacement oracle (on the CPU) must each
fail a pin: wrong stencil weights or denominator, a three-point formula, the
grid points out of order, a coupling factor with the wrong power."""
import numpy as np
import pytest

from oracle import mcpt_fd as F
from . import pins_fd

_orig_second = F.second_derivative
_orig_scaled = F.scaled


def _weights_15(e, h):
    em2, em1, e0, ep1, ep2 = (float(v) for v in e)
    return (-ep2 + 15.0 * ep1 - 28.0 * e0 + 15.0 * em1 - em2) / (12.0 * h * h)


def _denominator_6(e, h):
    return _orig_second(e, h) / 2.0


def _three_point(e, h):
    return (float(e[3]) - 2.0 * float(e[2]) + float(e[1])) / (h * h)


def _points_swapped(e, h):
    return _orig_second([e[1], e[0], e[2], e[3], e[4]], h)


def _square_power(prob, pairs, factors):
    return _orig_scaled(prob, pairs, np.asarray(factors) ** (2.0 / 3.0))


MUTATIONS = {
    "stencil_weights": ("second_derivative", _weights_15),
    "stencil_denominator": ("second_derivative", _denominator_6),
    "three_point_formula": ("second_derivative", _three_point),
    "grid_points_swapped": ("second_derivative", _points_swapped),
    "coupling_power": ("scaled", _square_power),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_fails_a_pin(name):
    attr, fn = MUTATIONS[name]
    orig = getattr(F, attr)
    setattr(F, attr, fn)
    try:
        results = {p.__name__: p(F) for p in pins_fd.ALL_FD_PINS}
    finally:
        setattr(F, attr, orig)
    failed = [k for k, (ok, _) in results.items() if not ok]
    assert failed, f"mutation {name} passed every pin"
