"""Brute-force twin of the reduced MCPT(2) equations, for tiny inputs only.

Written independently of the oracle: every two-electron integral is looked up
through a generic <pq|rs> = (pr|qs) function over the orbitals of the whole
cluster (real orbitals), so the index placement of each printed term of
Eqs. (58)-(59) follows from the paper's notation v^{pq}_{rs} alone; the dimer
amplitudes are solved for every ORDERED pair (the paper's dimer loop), without
assuming Tau_YX = Tau_XY^T.  Pure Python loops; o, v <= 3 or so.
"""
from __future__ import annotations

import numpy as np


class Orb:
    __slots__ = ("mono", "kind", "idx")

    def __init__(self, mono, kind, idx):
        self.mono, self.kind, self.idx = mono, kind, idx


class Cluster:
    def __init__(self, prob):
        self.prob = prob
        self.N = prob.n_mono
        self.occ = [[Orb(x, "o", i) for i in range(int(prob.n_occ[x]))] for x in range(self.N)]
        self.vir = [[Orb(x, "v", a) for a in range(int(prob.n_vir[x]))] for x in range(self.N)]
        self.eps = [np.asarray(prob.eps[prob.eps_off[x]:prob.eps_off[x + 1]]) for x in range(self.N)]
        self.pair_of = {}
        for p in range(prob.n_pair):
            x, y = (int(t) for t in prob.pairs[p])
            self.pair_of[(x, y)] = (p, False)
            self.pair_of[(y, x)] = (p, True)
        self.neighbours = [sorted(y for (x, y) in self.pair_of if x == m) for m in range(self.N)]

    def e(self, orb: Orb) -> float:
        o = int(self.prob.n_occ[orb.mono])
        return float(self.eps[orb.mono][orb.idx if orb.kind == "o" else o + orb.idx])

    def chem(self, p: Orb, r: Orb, q: Orb, s: Orb) -> float:
        """(pr|qs): electron 1 in p, r; electron 2 in q, s.  Only blocks with one
        occupied and one virtual orbital of the same monomer per electron are
        inputs; every other class is zero here."""
        if p.mono != r.mono or q.mono != s.mono:
            return 0.0
        if {p.kind, r.kind} != {"o", "v"} or {q.kind, s.kind} != {"o", "v"}:
            return 0.0
        i1, a1 = (p.idx, r.idx) if p.kind == "o" else (r.idx, p.idx)
        i2, a2 = (q.idx, s.idx) if q.kind == "o" else (s.idx, q.idx)
        x, y = p.mono, q.mono
        if x == y:
            return float(self.prob.k_of(x)[i1, i2, a1, a2])   # (a i|b j) = <ab|ij>
        if (x, y) not in self.pair_of:
            return 0.0
        pidx, rev = self.pair_of[(x, y)]
        V = self.prob.v_of(pidx)
        return float(V[i2, a2, i1, a1] if rev else V[i1, a1, i2, a2])

    def v(self, p, q, r, s) -> float:
        """v^{pq}_{rs} = <pq|rs> = (pr|qs)."""
        return self.chem(p, r, q, s)


SPINS = (0, 1)   # alpha, beta


def v_spin(cl: Cluster, p, sp, q, sq, r, sr, s, ss) -> float:
    """<p sp, q sq | r sr, s ss> between spin orbitals: the spatial (pr|qs) when
    electron 1 keeps its spin (sp == sr) and electron 2 keeps its spin (sq == ss)."""
    return cl.v(p, q, r, s) if (sp == sr and sq == ss) else 0.0


def pair_term(cl: Cluster, X: int, tau, i, i1, a, a1, sigma=0) -> float:
    """The pair term of Eq. (58) at (i, i1, a, a1) for the alpha electron pair
    (i, a) of X: the sum over every neighbour Y and every spin orbital k, c of Y
    (both spins: the spatial-orbital equation runs over spin orbitals there, and
    without exchange between monomers the dimer amplitude does not depend on
    the spin of Y's electron) of v^{a1 k}_{i1 c} Tau^{ac}_{ik} + v^{ak}_{ic} Tau^{a1 c}_{i1 k}."""
    s_ = 0.0
    for Y in cl.neighbours[X]:
        t = tau[(X, Y)]
        for k in cl.occ[Y]:
            for c in cl.vir[Y]:
                for sk in SPINS:
                    for sc in SPINS:
                        s_ += v_spin(cl, a1, sigma, k, sk, i1, sigma, c, sc) * t[i.idx, a.idx, k.idx, c.idx]
                        s_ += v_spin(cl, a, sigma, k, sk, i, sigma, c, sc) * t[i1.idx, a1.idx, k.idx, c.idx]
    return s_


def brute_tau(cl: Cluster, X: int, Y: int, T) -> np.ndarray:
    """Dimer amplitudes of the ordered pair (X, Y) from Eq. (59), reduced terms."""
    OX, VX, OY, VY = cl.occ[X], cl.vir[X], cl.occ[Y], cl.vir[Y]
    out = np.zeros((len(OX), len(VX), len(OY), len(VY)))
    for i in OX:
        for a in VX:
            for j in OY:
                for b in VY:
                    rhs = cl.v(a, b, i, j)                      # v^{ab}_{ij}
                    for i1 in OX:
                        for a1 in VX:                           # v^{i1 b}_{a1 j}(2T^{a a1}_{i i1} - T^{a a1}_{i1 i})
                            rhs += cl.v(i1, b, a1, j) * (2 * T[X][i.idx, i1.idx, a.idx, a1.idx]
                                                         - T[X][i1.idx, i.idx, a.idx, a1.idx])
                    for j1 in OY:
                        for b1 in VY:                           # v^{j1 a}_{b1 i}(2T^{b b1}_{j j1} - T^{b b1}_{j1 j})
                            rhs += cl.v(j1, a, b1, i) * (2 * T[Y][j.idx, j1.idx, b.idx, b1.idx]
                                                         - T[Y][j1.idx, j.idx, b.idx, b1.idx])
                    eps = cl.e(i) + cl.e(j) - cl.e(a) - cl.e(b)
                    out[i.idx, a.idx, j.idx, b.idx] = rhs / eps
    return out


def brute_T(cl: Cluster, X: int, tau) -> np.ndarray:
    """Monomer amplitudes from Eq. (58), source and pair terms; tau[(X, Y)] are
    the ordered-pair dimer amplitudes."""
    OX, VX = cl.occ[X], cl.vir[X]
    out = np.zeros((len(OX), len(OX), len(VX), len(VX)))
    for i in OX:
        for i1 in OX:
            for a in VX:
                for a1 in VX:
                    rhs = cl.v(a, a1, i, i1)                    # v^{a a1}_{i i1}
                    rhs += pair_term(cl, X, tau, i, i1, a, a1)
                    eps = cl.e(i) + cl.e(i1) - cl.e(a) - cl.e(a1)
                    out[i.idx, i1.idx, a.idx, a1.idx] = rhs / eps
    return out


def brute_energies(cl: Cluster, T, tau):
    e_m2 = []
    for X in range(cl.N):
        s = 0.0
        for i in cl.occ[X]:
            for i1 in cl.occ[X]:
                for a in cl.vir[X]:
                    for a1 in cl.vir[X]:
                        s += (2 * cl.v(i, i1, a, a1) - cl.v(i1, i, a, a1)) * T[X][i.idx, i1.idx, a.idx, a1.idx]
        e_m2.append(s)
    e_d2 = {}
    for (X, Y), t in tau.items():
        s = 0.0
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                for j in cl.occ[Y]:
                    for b in cl.vir[Y]:
                        s += 4 * cl.v(i, j, a, b) * t[i.idx, a.idx, j.idx, b.idx]
        e_d2[(X, Y)] = s
    return np.array(e_m2), e_d2


def brute_first_order(cl: Cluster):
    T = []
    for X in range(cl.N):
        OX, VX = cl.occ[X], cl.vir[X]
        t = np.zeros((len(OX), len(OX), len(VX), len(VX)))
        for i in OX:
            for i1 in OX:
                for a in VX:
                    for a1 in VX:
                        t[i.idx, i1.idx, a.idx, a1.idx] = cl.v(a, a1, i, i1) / (
                            cl.e(i) + cl.e(i1) - cl.e(a) - cl.e(a1))
        T.append(t)
    return T


def brute_sweeps(prob, n_sweeps: int, T0=None):
    """n_sweeps Jacobi sweeps from the first-order guess; returns T, ordered-pair
    Tau recomputed from the final T, and the energies."""
    cl = Cluster(prob)
    T = brute_first_order(cl) if T0 is None else [np.array(t) for t in T0]
    ordered = list(cl.pair_of.keys())
    for _ in range(n_sweeps):
        tau = {xy: brute_tau(cl, xy[0], xy[1], T) for xy in ordered}
        T = [brute_T(cl, X, tau) for X in range(cl.N)]
    tau = {xy: brute_tau(cl, xy[0], xy[1], T) for xy in ordered}
    e_m2, e_d2 = brute_energies(cl, T, tau)
    return T, tau, e_m2, e_d2


def dense_solve(prob):
    """Stack Eqs. (58)-(59) (reduced terms) for every T_X and every ordered-pair
    Tau as one linear system A x = b and solve it with LAPACK."""
    cl = Cluster(prob)
    index = {}
    n = 0
    for X in range(cl.N):
        for i in cl.occ[X]:
            for i1 in cl.occ[X]:
                for a in cl.vir[X]:
                    for a1 in cl.vir[X]:
                        index[("T", X, i.idx, i1.idx, a.idx, a1.idx)] = n
                        n += 1
    ordered = sorted(cl.pair_of.keys())
    for (X, Y) in ordered:
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                for j in cl.occ[Y]:
                    for b in cl.vir[Y]:
                        index[("U", X, Y, i.idx, a.idx, j.idx, b.idx)] = n
                        n += 1
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    for X in range(cl.N):
        for i in cl.occ[X]:
            for i1 in cl.occ[X]:
                for a in cl.vir[X]:
                    for a1 in cl.vir[X]:
                        row = index[("T", X, i.idx, i1.idx, a.idx, a1.idx)]
                        A[row, row] += cl.e(i) + cl.e(i1) - cl.e(a) - cl.e(a1)
                        rhs[row] += cl.v(a, a1, i, i1)
                        for Y in cl.neighbours[X]:
                            for k in cl.occ[Y]:
                                for c in cl.vir[Y]:
                                    for sk in SPINS:           # spin orbitals k, c of Y
                                        for sc in SPINS:
                                            A[row, index[("U", X, Y, i.idx, a.idx, k.idx, c.idx)]] -= \
                                                v_spin(cl, a1, 0, k, sk, i1, 0, c, sc)
                                            A[row, index[("U", X, Y, i1.idx, a1.idx, k.idx, c.idx)]] -= \
                                                v_spin(cl, a, 0, k, sk, i, 0, c, sc)
    for (X, Y) in ordered:
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                for j in cl.occ[Y]:
                    for b in cl.vir[Y]:
                        row = index[("U", X, Y, i.idx, a.idx, j.idx, b.idx)]
                        A[row, row] += cl.e(i) + cl.e(j) - cl.e(a) - cl.e(b)
                        rhs[row] += cl.v(a, b, i, j)
                        for i1 in cl.occ[X]:
                            for a1 in cl.vir[X]:
                                w = cl.v(i1, b, a1, j)
                                A[row, index[("T", X, i.idx, i1.idx, a.idx, a1.idx)]] -= 2 * w
                                A[row, index[("T", X, i1.idx, i.idx, a.idx, a1.idx)]] += w
                        for j1 in cl.occ[Y]:
                            for b1 in cl.vir[Y]:
                                w = cl.v(j1, a, b1, i)
                                A[row, index[("T", Y, j.idx, j1.idx, b.idx, b1.idx)]] -= 2 * w
                                A[row, index[("T", Y, j1.idx, j.idx, b.idx, b1.idx)]] += w
    x = np.linalg.solve(A, rhs)
    T = []
    for X in range(cl.N):
        o, v = int(prob.n_occ[X]), int(prob.n_vir[X])
        t = np.zeros((o, o, v, v))
        for key, r in index.items():
            if key[0] == "T" and key[1] == X:
                t[key[2:]] = x[r]
        T.append(t)
    tau = {}
    for (X, Y) in ordered:
        t = np.zeros((int(prob.n_occ[X]), int(prob.n_vir[X]), int(prob.n_occ[Y]), int(prob.n_vir[Y])))
        tau[(X, Y)] = t
    for key, r in index.items():
        if key[0] == "U":
            tau[(key[1], key[2])][key[3:]] = x[r]
    e_m2, e_d2 = brute_energies(cl, T, tau)
    return T, tau, e_m2, e_d2


def supersystem_mp2(prob) -> float:
    """Textbook closed-shell second-order energy of the whole cluster,
        E = sum_{IJAB} (IA|JB) [2 (IA|JB) - (IB|JA)] / (e_I + e_J - e_A - e_B),
    over all occupied I, J and virtual A, B of every monomer, with the cluster's
    integrals taken from the same generic lookup."""
    cl = Cluster(prob)
    occ = [o for X in range(cl.N) for o in cl.occ[X]]
    vir = [v for X in range(cl.N) for v in cl.vir[X]]
    e = 0.0
    for I in occ:
        for J in occ:
            for A in vir:
                for B in vir:
                    iajb = cl.chem(I, A, J, B)
                    if iajb == 0.0:
                        continue
                    ibja = cl.chem(I, B, J, A)
                    e += iajb * (2 * iajb - ibja) / (cl.e(I) + cl.e(J) - cl.e(A) - cl.e(B))
    return e


def brute_singles_first_order(cl: Cluster, w):
    """t^a_i = w^a_i / eps^i_a (the singles start of step 4, first order)."""
    t = []
    for X in range(cl.N):
        tx = np.zeros((len(cl.occ[X]), len(cl.vir[X])))
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                tx[i.idx, a.idx] = w[X][i.idx, a.idx] / (cl.e(i) - cl.e(a))
        t.append(tx)
    return t


def brute_singles_sweep(cl: Cluster, w, t):
    """One Jacobi sweep of Eq. (57), source and pair terms:
    eps^i_a t^a_i = w^a_i + sum over neighbours Y and spin orbitals k, c of Y of
    v^{ak}_{ic} t^c_k (closed shell: t^c_k is the same for both spins)."""
    out = []
    for X in range(cl.N):
        tx = np.zeros((len(cl.occ[X]), len(cl.vir[X])))
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                rhs = w[X][i.idx, a.idx]
                for Y in cl.neighbours[X]:
                    for k in cl.occ[Y]:
                        for c in cl.vir[Y]:
                            for sk in SPINS:
                                for sc in SPINS:                           # v^{ak}_{ic}, i, a alpha
                                    rhs += v_spin(cl, a, 0, k, sk, i, 0, c, sc) * t[Y][k.idx, c.idx]
                tx[i.idx, a.idx] = rhs / (cl.e(i) - cl.e(a))
        out.append(tx)
    return out


def brute_singles_energy(cl: Cluster, w, t):
    """E_M1(X) = 2 w^i_a t^a_i (Eq. 53), per monomer."""
    e = []
    for X in range(cl.N):
        s = 0.0
        for i in cl.occ[X]:
            for a in cl.vir[X]:
                s += 2.0 * w[X][i.idx, a.idx] * t[X][i.idx, a.idx]
        e.append(s)
    return np.array(e)
