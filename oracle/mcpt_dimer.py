"""Plain FP64 CPU oracle of the dimer-internal terms of the dimer doubles equation of MCPT(2).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and must never be called by the product.

What it computes (Byrd et al., "Molecular Cluster Perturbation Theory. I",
Sec. II.C, Eq. 59 (td2)): the terms of the dimer equation that act on the
dimer amplitudes Tau_XY themselves - the particle-particle ladder
v^{ab}_{a1 b1} Tau^{a1 b1}_{ij}, the hole-hole ladder v^{i1 j1}_{ij}
Tau^{ab}_{i1 j1}, the two cross rings -v^{b i1}_{b1 i} Tau^{a b1}_{i1 j} and
-v^{a j1}_{a1 j} Tau^{a1 b}_{i j1}, and the two monomer rings
(2 v^{i1 a}_{a1 i} - v^{a i1}_{a1 i}) Tau^{a1 b}_{i1 j} and
(2 v^{j1 b}_{b1 j} - v^{b j1}_{b1 j}) Tau^{a b1}_{i j1} - and the coupled
iteration of Eqs. 58 and 59 with them, in which Tau becomes an unknown of its
own.

Readings (in addition to those of mcpt_oracle and mcpt_lccd):

* Integral classes.  For a stored pair (X first) the dimer classes are
  W_XY[a,b,a1,b1] = <a b|a1 b1> = (a a1|b b1), Q_XY[i1,j1,i,j] = <i1 j1|i j> =
  (i1 i|j1 j), C_X[i1,i,b,b1] = (i1 i|b b1) and C_Y[j1,j,a,a1] = (j1 j|a a1),
  so v^{b i1}_{b1 i} = (b b1|i1 i) = C_X[i1,i,b,b1] and v^{a j1}_{a1 j} =
  (a a1|j1 j) = C_Y[j1,j,a,a1].  The monomer rings use the monomer classes:
  v^{i1 a}_{a1 i} = (a i|a1 i1) = K_X[i,i1,a,a1] and v^{a i1}_{a1 i} =
  (a a1|i1 i) = J_X[i1,i,a,a1] (likewise on Y).
* Sign: eps * Tau = v + (every printed term with its printed sign), as for
  the other terms.  With physical integrals and no exchange between the
  monomers this reproduces spin-orbital LCCD of the dimer restricted to the
  excitations that keep each electron on its monomer (pinned).
* Iteration: one coupled sweep takes Eq. 59 for every pair from the current T
  and the previous sweep's Tau (zero before the first sweep), then Eq. 58
  from the new Tau (Jacobi in both unknowns); the stopping test is the one on
  T.  The energies use the final T and the Tau of one more Eq. 59 step from
  it and the last Tau.
"""
from __future__ import annotations

import numpy as np

from . import mcpt_lccd as lccd
from . import mcpt_oracle as base


def internal_terms(W, Q, CX, CY, KX, JX, KY, JY, Tau) -> np.ndarray:
    """Sum of the dimer-internal terms of Eq. 59 for Tau[i, a, j, b] = Tau^{ab}_{ij}
    (i, a on X; j, b on Y), as a tensor [i, a, j, b]."""
    out = np.einsum("abAB,iAjB->iajb", W, Tau, optimize=True)          # v^{ab}_{a1 b1} Tau^{a1 b1}_{ij}
    out += np.einsum("IJij,IaJb->iajb", Q, Tau, optimize=True)         # v^{i1 j1}_{ij} Tau^{ab}_{i1 j1}
    out -= np.einsum("Iibc,Iajc->iajb", CX, Tau, optimize=True)        # v^{b i1}_{b1 i} Tau^{a b1}_{i1 j}
    out -= np.einsum("Jjac,icJb->iajb", CY, Tau, optimize=True)        # v^{a j1}_{a1 j} Tau^{a1 b}_{i j1}
    out += 2.0 * np.einsum("iIaA,IAjb->iajb", KX, Tau, optimize=True)  # 2 v^{i1 a}_{a1 i} Tau^{a1 b}_{i1 j}
    out -= np.einsum("Iiac,Icjb->iajb", JX, Tau, optimize=True)        # v^{a i1}_{a1 i} Tau^{a1 b}_{i1 j}
    out += 2.0 * np.einsum("jJbB,iaJB->iajb", KY, Tau, optimize=True)  # 2 v^{j1 b}_{b1 j} Tau^{a b1}_{i j1}
    out -= np.einsum("Jjbd,iaJd->iajb", JY, Tau, optimize=True)        # v^{b j1}_{b1 j} Tau^{a b1}_{i j1}
    return out


class DimerOracle(lccd.LccdOracle):
    """The full-monomer-equation oracle plus the dimer classes of each pair."""

    def __init__(self, prob, ints, dints):
        super().__init__(prob, ints)
        self.J = [np.asarray(ints.j_of(x), dtype=np.float64) for x in range(self.N)]
        self.dints = dints

    def internal(self, p, Tau_p):
        x, y = (int(t) for t in self.prob.pairs[p])
        d = self.dints
        f = lambda a: np.asarray(a, dtype=np.float64)
        return internal_terms(f(d.w_of(p)), f(d.q_of(p)), f(d.cx_of(p)), f(d.cy_of(p)),
                              self.K[x], self.J[x], self.K[y], self.J[y], Tau_p)

    def pair_phase(self, T, pairs=None, Tau_prev=None):
        """Tau of every stored pair from the current T and the previous Tau (Eq. 59)."""
        pairs = range(self.prob.n_pair) if pairs is None else pairs
        out = []
        for p in pairs:
            x, y = (int(t) for t in self.prob.pairs[p])
            Dp = self.D_pair(p)
            tau = base.dimer_amplitudes(self.V(p), T[x], T[y], Dp)
            if Tau_prev is not None:
                tau = tau + Dp * self.internal(p, Tau_prev[p])
            out.append(tau)
        return out


def solve(prob, ints, dints, tol: float = 1e-10, max_sweeps: int = 200, iso_tol: float | None = None,
          iso_max_sweeps: int | None = None) -> base.OracleResult:
    """Steps 5 and 6 with every term of Eqs. 58 and 59.  tol == 0 runs exactly
    max_sweeps coupled sweeps.  e_m2_0 holds E_LCCD(X) of step 5."""
    e_lccd, _, _, _ = lccd.isolated_lccd(prob, ints, tol if iso_tol is None else iso_tol,
                                         max_sweeps if iso_max_sweeps is None else iso_max_sweeps)
    orc = DimerOracle(prob, ints, dints)
    T = orc.first_order()
    Tau = [np.zeros_like(orc.D_pair(p)) for p in range(prob.n_pair)]
    residuals = []
    status = base.STATUS_NOT_CONVERGED if tol > 0 else base.STATUS_OK
    for _ in range(max_sweeps):
        Tau = orc.pair_phase(T, Tau_prev=Tau)
        T_new = orc.monomer_phase(Tau, T)
        r = max((float(np.max(np.abs(T_new[x] - T[x]))) for x in range(orc.N) if T[x].size), default=0.0)
        T = T_new
        residuals.append(r)
        if not np.isfinite(r):
            status = base.STATUS_DIVERGED
            break
        if tol > 0:
            if r < tol:
                status = base.STATUS_OK
                break
            if base.diverging(residuals):
                status = base.STATUS_DIVERGED
                break
    Tau = orc.pair_phase(T, Tau_prev=Tau)
    e_m2, e_d2 = orc.energies(T, Tau)
    return base.OracleResult(status, len(residuals), residuals, T, Tau, e_m2, e_lccd, e_d2)
