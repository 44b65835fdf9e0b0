"""Pins of the finite-displacement oracle (oracle.mcpt_fd) to facts outside itself.

Each pin takes the oracle module and returns (ok, detail); test_fd_pins.py runs
them on the real oracle and test_fd_mutations.py on broken copies."""
from __future__ import annotations

import numpy as np

from synth import central_cell, cubic_sites, displacement_scales, make_lattice_problem, stretch_modes
from .pins import TEST_WORKLOAD, _safe


@_safe
def pin_stencil_exact_on_quintics(orc):
    """The five-point second derivative is exact for every polynomial of degree
    at most five: f(x) = sum c_k x^k has f''(0) = 2 c_2."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for h in (0.01, 0.25, 1.0):
        for _ in range(5):
            c = rng.normal(size=6)
            f = [sum(c[k] * (s * h) ** k for k in range(6)) for s in (-2, -1, 0, 1, 2)]
            d = orc.second_derivative(f, h)
            worst = max(worst, abs(d - 2.0 * c[2]) / max(1.0, abs(2.0 * c[2])) * h * h)
    return worst < 1e-13, f"worst scaled error {worst:.3e}"


@_safe
def pin_stencil_order(orc):
    """For f = cos, the error of the five-point formula falls as h^4 (ratio 16
    when h halves) and is not exact (a sixth-degree term is present)."""
    e1 = abs(orc.second_derivative([np.cos(s * 0.2) for s in (-2, -1, 0, 1, 2)], 0.2) + 1.0)
    e2 = abs(orc.second_derivative([np.cos(s * 0.1) for s in (-2, -1, 0, 1, 2)], 0.1) + 1.0)
    return 14.0 < e1 / e2 < 18.0 and e2 > 0.0, f"error ratio {e1 / e2:.2f}"


@_safe
def pin_scaled_equals_displaced_geometry(orc):
    """A single monomer moved by s h along an axis: the oracle's scaled problem
    has exactly the blocks of the lattice generator's displaced geometry."""
    sites = cubic_sites(3, 2, 1)
    p = make_lattice_problem(sites, None, sizes=[(2, 3)] * 6, workload=TEST_WORKLOAD)
    worst = 0.0
    for mono, axis in ((0, 0), (3, 1), (4, 2)):
        e = np.zeros(3)
        e[axis] = 1.0
        pairs, f = displacement_scales(p, {mono: e}, step_angstrom=0.01)
        for k, s in enumerate((-2, -1, 1, 2)):
            q = orc.scaled(p, pairs, f[k])
            d = make_lattice_problem(sites, None, sizes=[(2, 3)] * 6, workload=TEST_WORKLOAD,
                                     displacement=(mono, axis, s * 0.01))
            worst = max(worst, float(np.max(np.abs(q.v - d.v)) / np.max(np.abs(d.v))))
    return worst < 1e-15, f"worst relative difference {worst:.3e}"


@_safe
def pin_step_independence(orc):
    """The second derivative of a small cluster's unit energy is the same at
    steps 0.01 and 0.005 A within the stencil's h^4 truncation and the
    convergence error amplified by 1 / h^2."""
    p = make_lattice_problem(cubic_sites(2, 2, 2), None, sizes=[(2, 3)] * 8, workload=TEST_WORKLOAD,
                             coupling_scale=3.0)
    cell = central_cell(p)
    d = []
    for h in (0.01, 0.005):
        name, pairs, f = stretch_modes(p, cell, step_angstrom=h)[0]
        d.append(orc.stencil(p, [(pairs, f)], cell, h, tol=1e-13)[0]["d2e"])
    return abs(d[0] - d[1]) < 1e-6 * abs(d[0]), f"{d[0]!r} vs {d[1]!r}"


ALL_FD_PINS = [pin_stencil_exact_on_quintics, pin_stencil_order, pin_scaled_equals_displaced_geometry,
               pin_step_independence]
