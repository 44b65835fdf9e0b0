"""Plain FP64 CPU oracle of the full monomer doubles equation of MCPT(2).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and must never be called by the product.

What it computes (Byrd et al., "Molecular Cluster Perturbation Theory. I",
Sec. II.C): the monomer doubles amplitudes of Eq. 58 (tm2) with every printed
term - the source, the intramonomer LCCD terms (particle-particle and
hole-hole ladders and the four ring combinations) and the pair coupling - and
the dimer amplitudes of Eq. 59 (td2) with the source and the monomer-amplitude
couplings; the isolated-monomer LCCD energies of step 5 of the program flow;
the coupled iteration of step 6; the energies E_M2 (Eq. 54), E_D2 (Eq. 55)
and the shift dE_M2 = E_M2 - E_LCCD (Eq. 56).

Readings (in addition to those of mcpt_oracle):

* Integral classes.  The intramonomer terms need, besides K_X[i,j,a,b] =
  <ab|ij>, the classes W_X[a,b,c,d] = <ab|cd>, Q_X[i,j,k,l] = <ij|kl> and
  J_X[i,j,a,b] = <ia|jb> = (ij|ab).  Each printed v^{pq}_{rs} = <pq|rs> =
  (pr|qs) is taken from them; with real orbitals (ai|jb) = (ai|bj), so the
  exchange-type ring integrals v^{a i2}_{i a2} and v^{i2 a}_{a2 i} are elements
  of K, and v^{a i2}_{a2 i} = (a a2|i2 i) = (i2 i|a a2) is an element of J.
* Sign: as for the reduced terms, eps * T = v + (every other printed term with
  its printed sign).  With physical integrals this reproduces spin-orbital
  LCCD (pinned).
* Step 5 (isolated LCCD) iterates the monomer equation without the pair term
  from the first-order guess with the same stopping rule; step 6 then starts
  again from the first-order guess.
* The dimer-internal terms of Eq. 59 need dimer integral classes that are not
  inputs and are not formed.
"""
from __future__ import annotations

import numpy as np

from . import mcpt_oracle as base


# ---------------------------------------------------------------------------
# the integrals by their names in Eq. 58
# ---------------------------------------------------------------------------
def named_integrals(K, J, W, Q) -> dict:
    """The intramonomer integrals of Eq. 58 as tensors indexed like the printed
    symbols, v^{pq}_{rs} -> [p, q, r, s]:

        vvvv[a, a1, a2, a3] = v^{a a1}_{a2 a3} = W[a, a1, a2, a3]
        oooo[i2, i3, i, i1] = v^{i2 i3}_{i i1} = Q[i2, i3, i, i1]
        voov[a, k, i, c]    = v^{a k}_{i c}  = (ai|kc) = (ai|ck) = K[i, k, a, c]
        vovo[a, k, c, i]    = v^{a k}_{c i}  = (ac|ki) = (ki|ac) = J[k, i, a, c]
        ovvo[k, a, c, i]    = v^{k a}_{c i}  = (kc|ai) = (ai|ck) = K[i, k, a, c]
    """
    return dict(vvvv=W, oooo=Q, voov=K.transpose(2, 1, 0, 3), vovo=J.transpose(2, 0, 3, 1),
                ovvo=K.transpose(1, 2, 3, 0))


def intramonomer_terms(v: dict, T: np.ndarray) -> np.ndarray:
    """Sum of the intramonomer terms of Eq. 58 for T[i, i1, a, a1] = T^{a a1}_{i i1}
    (index letters below: i, i1 -> i, j; a, a1 -> a, b; i2 -> k; a2 -> c):

        v^{a a1}_{a2 a3} T^{a2 a3}_{i i1}
      + v^{i2 i3}_{i i1} T^{a a1}_{i2 i3}
      + (v^{a i2}_{i a2} - v^{a i2}_{a2 i}) T^{a2 a1}_{i2 i1}
      + (v^{a1 i2}_{i1 a2} - v^{a1 i2}_{a2 i1}) T^{a2 a}_{i2 i}
      + v^{i2 a}_{a2 i} (T^{a2 a1}_{i2 i1} - T^{a2 a1}_{i1 i2})
      + v^{i2 a1}_{a2 i1} (T^{a2 a}_{i2 i} - T^{a2 a}_{i i2})
      - v^{a1 i2}_{a2 i} T^{a a2}_{i2 i1}
      - v^{a i2}_{a2 i1} T^{a1 a2}_{i2 i}
    """
    ring = v["voov"] - v["vovo"].transpose(0, 1, 3, 2)      # v^{a k}_{i c} - v^{a k}_{c i}, as [a, k, i, c]
    T_ex = T - T.transpose(1, 0, 2, 3)                     # T^{c b}_{k j} - T^{c b}_{j k}
    out = np.einsum("abcd,ijcd->ijab", v["vvvv"], T, optimize=True)
    out += np.einsum("klij,klab->ijab", v["oooo"], T, optimize=True)
    out += np.einsum("akic,kjcb->ijab", ring, T, optimize=True)
    out += np.einsum("bkjc,kica->ijab", ring, T, optimize=True)
    out += np.einsum("kaci,kjcb->ijab", v["ovvo"], T_ex, optimize=True)
    out += np.einsum("kbcj,kica->ijab", v["ovvo"], T_ex, optimize=True)
    out -= np.einsum("bkci,kjac->ijab", v["vovo"], T, optimize=True)
    out -= np.einsum("akcj,kibc->ijab", v["vovo"], T, optimize=True)
    return out


# ---------------------------------------------------------------------------
# step 5 and step 6
# ---------------------------------------------------------------------------
class LccdOracle(base.Oracle):
    """The reduced-term oracle plus the intramonomer integrals of each monomer."""

    def __init__(self, prob, ints):
        super().__init__(prob)
        self.v = [named_integrals(self.K[x], np.asarray(ints.j_of(x), dtype=np.float64),
                                  np.asarray(ints.w_of(x), dtype=np.float64),
                                  np.asarray(ints.q_of(x), dtype=np.float64)) for x in range(self.N)]

    def monomer_phase(self, Tau, T, monomers=None, couple=True):
        """New monomer amplitudes from Eq. 58: source, intramonomer terms of the
        current T, and (couple) the pair terms of the current Tau."""
        monomers = range(self.N) if monomers is None else monomers
        out = []
        for x in monomers:
            cs = [intramonomer_terms(self.v[x], T[x])]
            if couple:
                for p, first in self.nb[x]:
                    V = self.V(p)
                    if first:
                        cs.append(base.pair_coupling(V, Tau[p]))
                    else:
                        cs.append(base.pair_coupling(V.transpose(2, 3, 0, 1), Tau[p].transpose(2, 3, 0, 1)))
            out.append(base.monomer_amplitudes(self.K[x], self.D[x], cs))
        return out


def _iterate(step, T, n_mono, tol, max_sweeps):
    residuals = []
    status = base.STATUS_NOT_CONVERGED if tol > 0 else base.STATUS_OK
    for _ in range(max_sweeps):
        T_new = step(T)
        r = max((float(np.max(np.abs(T_new[x] - T[x]))) for x in range(n_mono) if T[x].size), default=0.0)
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
    return T, status, residuals


def isolated_lccd(prob, ints, tol: float = 1e-10, max_sweeps: int = 200):
    """Step 5: each monomer's LCCD without its environment, iterated from the
    first-order amplitudes until max|T_new - T| < tol.  Returns (E_LCCD per
    monomer, T, status, residuals)."""
    orc = LccdOracle(prob, ints)
    T, status, residuals = _iterate(lambda T: orc.monomer_phase(None, T, couple=False),
                                    orc.first_order(), orc.N, tol, max_sweeps)
    e = np.array([base.monomer_energy(orc.K[x], T[x]) for x in range(orc.N)])
    return e, T, status, residuals


def solve(prob, ints, tol: float = 1e-10, max_sweeps: int = 200, iso_tol: float | None = None,
          iso_max_sweeps: int | None = None) -> base.OracleResult:
    """Steps 5 and 6.  One coupled sweep = Eq. 59 for every pair from the current
    T, then Eq. 58 (source, intramonomer terms of the current T, pair terms) for
    every monomer.  tol == 0 runs exactly max_sweeps coupled sweeps.  The
    result's e_m2_0 holds E_LCCD(X) of step 5 (so de_m2 is Eq. 56)."""
    e_lccd, _, _, _ = isolated_lccd(prob, ints, tol if iso_tol is None else iso_tol,
                                    max_sweeps if iso_max_sweeps is None else iso_max_sweeps)
    orc = LccdOracle(prob, ints)

    def sweep(T):
        return orc.monomer_phase(orc.pair_phase(T), T)

    T, status, residuals = _iterate(sweep, orc.first_order(), orc.N, tol, max_sweeps)
    Tau = orc.pair_phase(T)
    e_m2, e_d2 = orc.energies(T, Tau)
    return base.OracleResult(status, len(residuals), residuals, T, Tau, e_m2, e_lccd, e_d2)
