"""Plain FP64 CPU oracle of the MCPT(2) singles iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and must never be called by the product.

What it computes (Byrd et al., "Molecular Cluster Perturbation Theory. I",
Sec. II.C): the monomer singles amplitudes t^a_i of Eq. 57 (tm1), iterated to
self-consistency as in step 4 of the program flow, and the singles energy
E_M1(X) = 2 w^i_a t^a_i of Eq. 53 (em1).

Readings taken where the paper is silent or ambiguous:

* Terms kept: the one-electron embedding source w^a_i and the pair coupling
  sum over neighbours Y of v^{ak}_{ic} t^c_k; and, when the intramonomer
  integral classes are given (the full monomer equation's inputs), the
  intramonomer term (2 v^{a i1}_{i a1} - v^{a i}_{a1 i1}) t^{a1}_{i1} with
  v^{a i1}_{i a1} = (ai|i1 a1) = K[i, i1, a, a1] (real orbitals) and
  v^{a i}_{a1 i1} = (a a1|i i1) = J[i, i1, a, a1].  Without them the term is
  dropped as a whole: it pairs an ov|ov integral with an oo|vv one, and keeping
  half of it would be an arbitrary truncation (the rule of the doubles).
* Sign: eps^i_a t = w + (the printed coupling with its printed sign), with
  eps^i_a = e_i - e_a, i.e. t = d * (w + 2 sum_Y v t), d = 1 / (e_i - e_a); the
  same reading as the doubles.  At zero coupling the energy is then
  2 sum |w|^2 / (e_i - e_a) < 0, the textbook second-order singles energy.
* v^{ak}_{ic} with i, a on X and k, c on Y is (ai|ck) = V_XY[i, a, k, c], the
  Coulomb block the doubles use; for the reversed pair it is V_XY transposed.
* Spin sum: as for the pair term of Eq. 58, the summed k, c of Y run over both
  spins (the intramonomer term's 2v has the same origin), so the pair sum
  carries a factor 2: t = d * (w + 2 sum_Y v t).  Pinned against restricted
  spin-orbital linear singles on a dimer cut from one real two-electron tensor.
* One sweep updates every monomer from the previous amplitudes (Jacobi); the
  initial guess is the first-order amplitude t = d * w (step 4 starts from w);
  the residual is max |t_new - t| over all monomers; the divergence rule is the
  doubles' one.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .mcpt_oracle import SPIN_SUM, STATUS_DIVERGED, STATUS_NOT_CONVERGED, STATUS_OK, diverging


def singles_denominator(e_occ: np.ndarray, e_vir: np.ndarray) -> np.ndarray:
    """d[i, a] = 1 / (e_i - e_a)  (eps^i_a of Eq. 57, Eqs. 60-61 with one pair of indices)."""
    return 1.0 / (e_occ[:, None] - e_vir[None, :])


def singles_energy(w: np.ndarray, t: np.ndarray) -> float:
    """E_M1(X) = 2 w^i_a t^a_i  (Eq. 53)."""
    return 2.0 * float(np.sum(w * t))


@dataclasses.dataclass
class SinglesResult:
    status: int
    sweeps: int
    residuals: list
    t: list
    e_m1: np.ndarray
    e_m1_0: np.ndarray

    @property
    def e_total(self) -> float:
        return float(np.sum(self.e_m1))

    @property
    def e_total0(self) -> float:
        return float(np.sum(self.e_m1_0))


def _split(prob, w):
    w = np.asarray(w, dtype=np.float64)
    out, off = [], 0
    for x in range(prob.n_mono):
        o, v = int(prob.n_occ[x]), int(prob.n_vir[x])
        out.append(w[off:off + o * v].reshape(o, v))
        off += o * v
    return out


def coupling(prob, t):
    """u_X = 2 sum over the neighbours Y of X of v^{ak}_{ic} t^c_k  (the pair sum of
    Eq. 57, summed over both spins of k, c)."""
    u = [np.zeros_like(tx) for tx in t]
    for p in range(prob.n_pair):
        x, y = (int(q) for q in prob.pairs[p])
        V = np.asarray(prob.v_of(p), dtype=np.float64)          # [i, a, k, c], i, a on X
        u[x] += np.einsum("iakc,kc->ia", V, t[y])
        u[y] += np.einsum("iakc,ia->kc", V, t[x])               # reversed pair: V_XY transposed
    return [SPIN_SUM * ux for ux in u]


def intramonomer(K: np.ndarray, J: np.ndarray, t: np.ndarray) -> np.ndarray:
    """(2 v^{a i1}_{i a1} - v^{a i}_{a1 i1}) t^{a1}_{i1} of Eq. 57 as [i, a], with
    v^{a i1}_{i a1} = K[i, i1, a, a1] and v^{a i}_{a1 i1} = J[i, i1, a, a1]."""
    return np.einsum("IJAB,JB->IA", 2.0 * K - J, t)


def solve(prob, w, tol: float = 1e-10, max_sweeps: int = 500, ints=None) -> SinglesResult:
    """Iterate t = d * (w + 2 sum_Y v t [+ intramonomer term]) until
    max |t_new - t| < tol (tol == 0: exactly max_sweeps sweeps, status OK unless
    the residual became non-finite).  ints: the intramonomer integral classes
    (an object with j_of(x) = J_X[i, j, a, b] = (ij|ab)), or None."""
    ws = _split(prob, w)
    d = [singles_denominator(*prob.eps_of(x)) for x in range(prob.n_mono)]
    t = [d[x] * ws[x] for x in range(prob.n_mono)]
    e0 = np.array([singles_energy(ws[x], t[x]) for x in range(prob.n_mono)])
    KJ = None if ints is None else [(np.asarray(prob.k_of(x), dtype=np.float64),
                                     np.asarray(ints.j_of(x), dtype=np.float64)) for x in range(prob.n_mono)]
    residuals = []
    status = STATUS_NOT_CONVERGED if tol > 0 else STATUS_OK
    sweeps = 0
    for _ in range(max_sweeps):
        u = coupling(prob, t)
        if KJ is not None:
            u = [u[x] + intramonomer(KJ[x][0], KJ[x][1], t[x]) for x in range(prob.n_mono)]
        t_new = [d[x] * (ws[x] + u[x]) for x in range(prob.n_mono)]
        r = max((float(np.max(np.abs(t_new[x] - t[x]))) for x in range(prob.n_mono) if t[x].size),
                default=0.0)
        t = t_new
        sweeps += 1
        residuals.append(r)
        if not np.isfinite(r):
            status = STATUS_DIVERGED
            break
        if tol > 0:
            if r < tol:
                status = STATUS_OK
                break
            if diverging(residuals):
                status = STATUS_DIVERGED
                break
    e = np.array([singles_energy(ws[x], t[x]) for x in range(prob.n_mono)])
    return SinglesResult(status, sweeps, residuals, t, e, e0)
