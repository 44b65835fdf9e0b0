"""Plain FP64 CPU oracle of the MCPT(2) doubles iteration.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this module.  It shares no code with the HIP path
and must never be called by the product.

What it computes (Byrd et al., "Molecular Cluster Perturbation Theory. I",
Sec. II.C): the monomer doubles amplitudes T_X (Eq. 58, tm2) and the dimer
doubles amplitudes Tau_XY (Eq. 59, td2), iterated to self-consistency (program
flow, step 6), and the energies E_M2(X) (Eq. 54, em2), E_D2(XY) (Eq. 55, ed2)
and the shift dE_M2(X) (Eq. 56, dem2).

Readings taken where the paper is silent, garbled or ambiguous:

* Only the terms that the supplied integral classes can form are kept: the
  source terms v^{aa1}_{ii1} and v^{ab}_{ij}, the pair coupling of Eq. 58
  (sum over Y of v.Tau) and the monomer-amplitude coupling of Eq. 59
  (v (2T - T)).  The intramonomer LCCD terms of Eq. 58 and the dimer-internal
  terms of Eq. 59 need integral classes that are not inputs.
* Sign: each amplitude equation is read as  eps * T = v + (the other printed
  terms with their printed signs), i.e. T = D * (v + ...), with
  eps^{ij}_{ab} = e_i + e_j - e_a - e_b and D = 1/eps (Eqs. 60-61).  At zero
  coupling this gives the (negative) closed-shell second-order energy.
* Spin sum of the pair term.  The printed pair term of Eq. 58 carries no spin
  factor, while every other Coulomb loop of the spin-adapted equations does
  (the 2v - v rings, the 2T - T of Eq. 59, the 2v of the embedding field of
  Eq. 26).  Sec. II.A states that the method is LCCD for canonical HF orbitals;
  on integrals cut from one real two-electron tensor of a dimer without
  exchange between the monomers, restricted spin-orbital LCCD reproduces the
  spatial-orbital equations exactly when the summed k, c of Y run over both
  spins, which doubles the printed term.  The oracle therefore carries the
  factor 2 (the spin-summed reading); the printed half is a planted mistake
  that the pins reject.
* Every o.v.o.v dimer integral in Eqs. 55, 58 and 59 is the one Coulomb block
  V_XY[i, a, j, b] = (ai|bj) of real orbitals (Eq. 29 with i, a on X and j, b
  on Y); the block of the reversed pair is its transpose.
* Each unordered pair is stored and solved once; Tau_YX is Tau_XY transposed
  (the theory is Hermitian, Sec. II.A), and E_dimer sums E_D2 over unordered
  pairs.
* One sweep = all dimer amplitudes from the current T (Eq. 59), then all
  monomer amplitudes from those Tau (Eq. 58); the initial guess is the
  first-order amplitude T = D * v (step 6 uses the integrals as the guess).
  The residual is the max-norm of the change of T; energies are evaluated from
  the final T and the Tau recomputed from it.
* The isolated-monomer reference of Eq. 56 is the zero-coupling energy of the
  same reduced equations, E_M2 at T = D * K.
"""
from __future__ import annotations

import dataclasses

import numpy as np


# ---------------------------------------------------------------------------
# denominators, Eqs. (60)-(61)
# ---------------------------------------------------------------------------
def monomer_denominator(e_occ: np.ndarray, e_vir: np.ndarray) -> np.ndarray:
    """D[i, j, a, b] = 1 / (e_i + e_j - e_a - e_b), all indices on one monomer."""
    ei = e_occ[:, None, None, None]
    ej = e_occ[None, :, None, None]
    ea = e_vir[None, None, :, None]
    eb = e_vir[None, None, None, :]
    return 1.0 / (ei + ej - ea - eb)


def pair_denominator(ex_occ, ex_vir, ey_occ, ey_vir) -> np.ndarray:
    """D[i, a, j, b] = 1 / (e_i + e_j - e_a - e_b) with i, a on X and j, b on Y."""
    ei = ex_occ[:, None, None, None]
    ea = ex_vir[None, :, None, None]
    ej = ey_occ[None, None, :, None]
    eb = ey_vir[None, None, None, :]
    return 1.0 / (ei + ej - ea - eb)


# ---------------------------------------------------------------------------
# energies, Eqs. (54)-(56)
# ---------------------------------------------------------------------------
def monomer_energy(K: np.ndarray, T: np.ndarray) -> float:
    """E_M2(X) = (2 v^{i i1}_{a a1} - v^{i1 i}_{a a1}) T^{a a1}_{i i1}  (Eq. 54).

    K[i, i1, a, a1] = <a a1|i i1>; for real orbitals v^{i i1}_{a a1} is the
    same number and v^{i1 i}_{a a1} = K[i1, i, a, a1]."""
    v_direct = K
    v_exch = K.transpose(1, 0, 2, 3)
    return float(np.einsum("ijab,ijab->", 2.0 * v_direct - v_exch, T))


def dimer_energy(V: np.ndarray, Tau: np.ndarray) -> float:
    """E_D2(XY) = 4 v^{ij}_{ab} Tau^{ab}_{ij}  (Eq. 55); v^{ij}_{ab} = V[i, a, j, b]."""
    return 4.0 * float(np.einsum("iajb,iajb->", V, Tau))


# ---------------------------------------------------------------------------
# amplitude equations, Eqs. (58)-(59), reduced terms
# ---------------------------------------------------------------------------
def spin_adapted(T: np.ndarray) -> np.ndarray:
    """(2 T^{a a1}_{i i1} - T^{a a1}_{i1 i}) as a tensor [i, i1, a, a1] (Eq. 59)."""
    return 2.0 * T - T.transpose(1, 0, 2, 3)


def dimer_amplitudes(V: np.ndarray, T_x: np.ndarray, T_y: np.ndarray, D_xy: np.ndarray) -> np.ndarray:
    """Tau^{ab}_{ij} from Eq. (59), source and monomer-amplitude couplings:

        eps Tau = v^{ab}_{ij}
                + v^{i1 b}_{a1 j} (2 T^{a a1}_{i i1} - T^{a a1}_{i1 i})      (T of X)
                + v^{j1 a}_{b1 i} (2 T^{b b1}_{j j1} - T^{b b1}_{j1 j})      (T of Y)

    with v^{i1 b}_{a1 j} = (a1 i1|b j) = V[i1, a1, j, b] and
    v^{j1 a}_{b1 i} = (a i|b1 j1) = V[i, a, j1, b1]."""
    src = V
    from_x = np.einsum("IAjb,iIaA->iajb", V, spin_adapted(T_x), optimize=True)
    from_y = np.einsum("iaJB,jJbB->iajb", V, spin_adapted(T_y), optimize=True)
    return D_xy * (src + from_x + from_y)


SPIN_SUM = 2.0   # both spins of the summed k, c on Y (Sec. II.A: the method is LCCD)


def pair_coupling(V: np.ndarray, Tau: np.ndarray) -> np.ndarray:
    """The pair term of Eq. (58) for one neighbour Y of X, as a tensor [i, i1, a, a1]:

        2 (v^{a1 k}_{i1 c} Tau^{a c}_{i k} + v^{a k}_{i c} Tau^{a1 c}_{i1 k})

    with c, k on Y, v^{a1 k}_{i1 c} = V[i1, a1, k, c], Tau^{ac}_{ik} = Tau[i, a, k, c];
    the factor 2 is the sum over the two spins of the spatial k, c on Y."""
    t1 = np.einsum("IAkc,iakc->iIaA", V, Tau, optimize=True)
    t2 = np.einsum("iakc,IAkc->iIaA", V, Tau, optimize=True)
    return SPIN_SUM * (t1 + t2)


def monomer_amplitudes(K: np.ndarray, D_x: np.ndarray, couplings) -> np.ndarray:
    """T^{a a1}_{i i1} from Eq. (58): eps T = v^{a a1}_{i i1} + sum over Y of the
    (spin-summed) pair term."""
    rhs = K.copy()
    for c in couplings:
        rhs = rhs + c
    return D_x * rhs


# ---------------------------------------------------------------------------
# the iteration (program flow, step 6)
# ---------------------------------------------------------------------------
STATUS_OK = 0
STATUS_NOT_CONVERGED = -4
STATUS_DIVERGED = -5


@dataclasses.dataclass
class OracleResult:
    status: int
    sweeps: int
    residuals: list
    T: list
    Tau: list
    e_m2: np.ndarray
    e_m2_0: np.ndarray
    e_d2: np.ndarray

    @property
    def de_m2(self) -> np.ndarray:
        return self.e_m2 - self.e_m2_0

    @property
    def e_mono(self) -> float:
        return float(np.sum(self.e_m2))

    @property
    def e_dimer(self) -> float:
        return float(np.sum(self.e_d2))

    @property
    def e_total(self) -> float:
        return self.e_mono + self.e_dimer

    @property
    def e_mono0(self) -> float:
        return float(np.sum(self.e_m2_0))


class Oracle:
    """Holds per-monomer denominators and the oriented pair views of a problem."""

    def __init__(self, prob):
        self.prob = prob
        self.N = prob.n_mono
        self.eo, self.ev, self.K, self.D = [], [], [], []
        for x in range(self.N):
            eo, ev = prob.eps_of(x)
            self.eo.append(np.asarray(eo, dtype=np.float64))
            self.ev.append(np.asarray(ev, dtype=np.float64))
            self.K.append(np.asarray(prob.k_of(x), dtype=np.float64))
            self.D.append(monomer_denominator(self.eo[x], self.ev[x]))
        # neighbours of each monomer: (pair index, True if X is stored first)
        self.nb = [[] for _ in range(self.N)]
        for p in range(prob.n_pair):
            x, y = (int(t) for t in prob.pairs[p])
            self.nb[x].append((p, True))
            self.nb[y].append((p, False))

    def V(self, p):
        return np.asarray(self.prob.v_of(p), dtype=np.float64)

    def D_pair(self, p):
        x, y = (int(t) for t in self.prob.pairs[p])
        return pair_denominator(self.eo[x], self.ev[x], self.eo[y], self.ev[y])

    def first_order(self):
        return [self.D[x] * self.K[x] for x in range(self.N)]

    def pair_phase(self, T, pairs=None):
        """Tau of every stored pair from the current monomer amplitudes (Eq. 59)."""
        pairs = range(self.prob.n_pair) if pairs is None else pairs
        out = []
        for p in pairs:
            x, y = (int(t) for t in self.prob.pairs[p])
            out.append(dimer_amplitudes(self.V(p), T[x], T[y], self.D_pair(p)))
        return out

    def monomer_phase(self, Tau, monomers=None):
        """New monomer amplitudes from the dimer amplitudes (Eq. 58)."""
        monomers = range(self.N) if monomers is None else monomers
        out = []
        for x in monomers:
            cs = []
            for p, first in self.nb[x]:
                V = self.V(p)
                if first:
                    cs.append(pair_coupling(V, Tau[p]))
                else:   # reversed pair: V_XY = V_YX^T, Tau_XY = Tau_YX^T
                    cs.append(pair_coupling(V.transpose(2, 3, 0, 1), Tau[p].transpose(2, 3, 0, 1)))
            out.append(monomer_amplitudes(self.K[x], self.D[x], cs))
        return out

    def energies(self, T, Tau):
        e_m2 = np.array([monomer_energy(self.K[x], T[x]) for x in range(self.N)])
        e_d2 = np.array([dimer_energy(self.V(p), Tau[p]) for p in range(self.prob.n_pair)])
        return e_m2, e_d2


def diverging(residuals) -> bool:
    """Divergence rule: a non-finite residual, a residual above 1e6 times the
    first one, or three consecutive increases ending above the first one."""
    r = residuals[-1]
    if not np.isfinite(r):
        return True
    if r > 1e6 * residuals[0]:
        return True
    if len(residuals) >= 4 and residuals[-1] > residuals[-2] > residuals[-3] > residuals[-4] \
            and r > residuals[0]:
        return True
    return False


def solve(prob, tol: float = 1e-10, max_sweeps: int = 200, T0=None) -> OracleResult:
    """Iterate sweeps until max|T_new - T| < tol.

    tol == 0 runs exactly max_sweeps sweeps with no convergence test (fixed
    sweep count); the status is then OK unless the residual became non-finite."""
    orc = Oracle(prob)
    first = orc.first_order()
    e_m2_0 = np.array([monomer_energy(orc.K[x], first[x]) for x in range(orc.N)])
    T = [np.array(t, dtype=np.float64).reshape(first[x].shape) for x, t in enumerate(T0)] \
        if T0 is not None else first
    residuals = []
    status = STATUS_NOT_CONVERGED if tol > 0 else STATUS_OK
    sweeps = 0
    for _ in range(max_sweeps):
        Tau = orc.pair_phase(T)
        T_new = orc.monomer_phase(Tau)
        r = max((float(np.max(np.abs(T_new[x] - T[x]))) for x in range(orc.N) if T[x].size),
                default=0.0)
        T = T_new
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
    Tau = orc.pair_phase(T)
    e_m2, e_d2 = orc.energies(T, Tau)
    return OracleResult(status, sweeps, residuals, T, Tau, e_m2, e_m2_0, e_d2)
