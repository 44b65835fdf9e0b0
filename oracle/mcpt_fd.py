"""Plain FP64 CPU oracle of the finite-displacement workflow of MCPT(2).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and must never be called by the product.

What it computes (Byrd et al., "Molecular Cluster Perturbation Theory. I",
Sec. IV.A): harmonic force constants of stretch modes from single-point
energies on a five-point grid of displacements, each single point being the
additive unit energy of Eq. 66 over the monomers of a unit cell,
E = sum_X (E_SCF(X) + E_M1(X) + E_M2(X)).

Readings:

* A displaced geometry keeps the monomer integrals and the undisplaced pair
  list and rescales the dimer couplings of the moved monomers by (R0 / R)^3
  (the coupling model of the synthetic crystal); E_SCF(X) does not change
  under such displacements and is left out of the unit energy.
* Every single point is an independent converged solve (here from the
  first-order start; the GPU driver starts displaced points from the base
  amplitudes, which changes only the sweep count).
* The second derivative is the central five-point formula, exact for
  polynomials up to degree five (pinned).
"""
from __future__ import annotations

import numpy as np

from . import mcpt_oracle, mcpt_singles

GRID = (-2, -1, 0, 1, 2)


def second_derivative(e, h: float) -> float:
    """f''(0) from f at -2h, -h, 0, h, 2h: the Taylor expansions of f(+-h) and
    f(+-2h) about 0, combined so that the f(0), f'''' and odd terms cancel:
        (-f(2h) + 16 f(h) - 30 f(0) + 16 f(-h) - f(-2h)) / (12 h^2)."""
    em2, em1, e0, ep1, ep2 = (float(v) for v in e)
    return (-ep2 + 16.0 * ep1 - 30.0 * e0 + 16.0 * em1 - em2) / (12.0 * h * h)


def scaled(prob, pairs, factors):
    """The displaced problem: listed pair blocks multiplied by their factors."""
    from synth import scaled_problem
    return scaled_problem(prob, pairs, factors)


def unit_energy(prob, cell, tol: float, w=None, max_sweeps: int = 400):
    """Eq. 66 over the cell monomers (E_M2 and, with a singles source, E_M1)."""
    r = mcpt_oracle.solve(prob, tol=tol, max_sweeps=max_sweeps)
    if r.status != 0:
        raise RuntimeError(f"doubles status {r.status}")
    e = float(np.sum(r.e_m2[np.asarray(cell)]))
    if w is not None:
        s = mcpt_singles.solve(prob, w, tol=tol, max_sweeps=max_sweeps)
        if s.status != 0:
            raise RuntimeError(f"singles status {s.status}")
        e += float(np.sum(np.asarray(s.e_m1)[np.asarray(cell)]))
    return e, r.sweeps


def stencil(prob, modes, cell, h: float, tol: float = 1e-12, w=None):
    """For each mode (pairs, factors[4][n] at -2h, -h, +h, +2h): the five unit
    energies and the second derivative."""
    e0, _ = unit_energy(prob, cell, tol, w)
    out = []
    for pairs, factors in modes:
        e = [0.0] * 5
        e[2] = e0
        for k, slot in enumerate((0, 1, 3, 4)):
            e[slot], _ = unit_energy(scaled(prob, pairs, factors[k]), cell, tol, w)
        out.append({"e": e, "d2e": second_derivative(e, h)})
    return out
