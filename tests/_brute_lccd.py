"""Brute-force twin of the full monomer equation (Eq. 58 with its intramonomer
terms), for tiny inputs only.

Written independently of the oracle: every integral comes from a generic
(pr|qs) lookup over the orbitals of the cluster, and each printed term of
Eq. 58 is a loop over the printed indices with v^{pq}_{rs} = (pr|qs).  Dimer
amplitudes come from the reduced-term twin (ordered pairs).  Pure Python loops.
"""
from __future__ import annotations

import numpy as np

from . import _brute


class LccdCluster(_brute.Cluster):
    def __init__(self, prob, ints):
        super().__init__(prob)
        self.ints = ints

    def chem(self, p, r, q, s) -> float:
        """(pr|qs) with the intramonomer classes (vv|vv), (oo|oo), (oo|vv) of
        the integral set added to the ov|ov blocks of the reduced twin."""
        kinds = (p.kind, r.kind, q.kind, s.kind)
        if p.mono == r.mono == q.mono == s.mono:
            x = p.mono
            if kinds == ("v", "v", "v", "v"):      # (ac|bd) = <ab|cd> = W[a, b, c, d]
                return float(self.ints.w_of(x)[p.idx, q.idx, r.idx, s.idx])
            if kinds == ("o", "o", "o", "o"):      # (ik|jl) = <ij|kl> = Q[i, j, k, l]
                return float(self.ints.q_of(x)[p.idx, q.idx, r.idx, s.idx])
            if kinds == ("o", "o", "v", "v"):      # (ij|ab) = J[i, j, a, b]
                return float(self.ints.j_of(x)[p.idx, r.idx, q.idx, s.idx])
            if kinds == ("v", "v", "o", "o"):      # (ab|ij) = (ij|ab)
                return float(self.ints.j_of(x)[q.idx, s.idx, p.idx, r.idx])
        return super().chem(p, r, q, s)


def intramonomer(cl: LccdCluster, X: int, T, i, i1, a, a1) -> float:
    """The intramonomer terms of Eq. 58 at (i, i1, a, a1), term by term as printed."""
    O, V = cl.occ[X], cl.vir[X]
    t = T[X]
    s = 0.0
    for a2 in V:
        for a3 in V:                                  # v^{a a1}_{a2 a3} T^{a2 a3}_{i i1}
            s += cl.v(a, a1, a2, a3) * t[i.idx, i1.idx, a2.idx, a3.idx]
    for i2 in O:
        for i3 in O:                                  # v^{i2 i3}_{i i1} T^{a a1}_{i2 i3}
            s += cl.v(i2, i3, i, i1) * t[i2.idx, i3.idx, a.idx, a1.idx]
    for i2 in O:
        for a2 in V:
            # (v^{a i2}_{i a2} - v^{a i2}_{a2 i}) T^{a2 a1}_{i2 i1}
            s += (cl.v(a, i2, i, a2) - cl.v(a, i2, a2, i)) * t[i2.idx, i1.idx, a2.idx, a1.idx]
            # (v^{a1 i2}_{i1 a2} - v^{a1 i2}_{a2 i1}) T^{a2 a}_{i2 i}
            s += (cl.v(a1, i2, i1, a2) - cl.v(a1, i2, a2, i1)) * t[i2.idx, i.idx, a2.idx, a.idx]
            # v^{i2 a}_{a2 i} (T^{a2 a1}_{i2 i1} - T^{a2 a1}_{i1 i2})
            s += cl.v(i2, a, a2, i) * (t[i2.idx, i1.idx, a2.idx, a1.idx] - t[i1.idx, i2.idx, a2.idx, a1.idx])
            # v^{i2 a1}_{a2 i1} (T^{a2 a}_{i2 i} - T^{a2 a}_{i i2})
            s += cl.v(i2, a1, a2, i1) * (t[i2.idx, i.idx, a2.idx, a.idx] - t[i.idx, i2.idx, a2.idx, a.idx])
            # - v^{a1 i2}_{a2 i} T^{a a2}_{i2 i1}
            s -= cl.v(a1, i2, a2, i) * t[i2.idx, i1.idx, a.idx, a2.idx]
            # - v^{a i2}_{a2 i1} T^{a1 a2}_{i2 i}
            s -= cl.v(a, i2, a2, i1) * t[i2.idx, i.idx, a1.idx, a2.idx]
    return s


def brute_T_full(cl: LccdCluster, X: int, T, tau, couple=True) -> np.ndarray:
    """Eq. 58 with every printed term; tau[(X, Y)]: ordered-pair dimer amplitudes."""
    O, V = cl.occ[X], cl.vir[X]
    out = np.zeros((len(O), len(O), len(V), len(V)))
    for i in O:
        for i1 in O:
            for a in V:
                for a1 in V:
                    rhs = cl.v(a, a1, i, i1) + intramonomer(cl, X, T, i, i1, a, a1)
                    if couple:
                        rhs += _brute.pair_term(cl, X, tau, i, i1, a, a1)
                    out[i.idx, i1.idx, a.idx, a1.idx] = rhs / (cl.e(i) + cl.e(i1) - cl.e(a) - cl.e(a1))
    return out


def brute_lccd_sweeps(prob, ints, n_iso: int, n_sweeps: int):
    """n_iso isolated sweeps (step 5) -> E_LCCD per monomer; then n_sweeps coupled
    sweeps (step 6) from the first-order guess; Tau from the final T; energies."""
    cl = LccdCluster(prob, ints)
    T = _brute.brute_first_order(cl)
    for _ in range(n_iso):
        T = [brute_T_full(cl, X, T, None, couple=False) for X in range(cl.N)]
    e_iso, _ = _brute.brute_energies(cl, T, {})
    T = _brute.brute_first_order(cl)
    ordered = list(cl.pair_of.keys())
    for _ in range(n_sweeps):
        tau = {xy: _brute.brute_tau(cl, xy[0], xy[1], T) for xy in ordered}
        T = [brute_T_full(cl, X, T, tau) for X in range(cl.N)]
    tau = {xy: _brute.brute_tau(cl, xy[0], xy[1], T) for xy in ordered}
    e_m2, e_d2 = _brute.brute_energies(cl, T, tau)
    return T, tau, e_m2, e_d2, e_iso


def dense_lccd(prob, ints):
    """The converged fixed point as a dense linear system over every T_X element
    and every ordered-pair Tau element, assembled term by term from the printed
    equations by probing each unknown, and solved with LAPACK."""
    cl = LccdCluster(prob, ints)
    shapes_T = [(int(prob.n_occ[X]),) * 2 + (int(prob.n_vir[X]),) * 2 for X in range(cl.N)]
    ordered = sorted(cl.pair_of.keys())
    shapes_U = [(int(prob.n_occ[X]), int(prob.n_vir[X]), int(prob.n_occ[Y]), int(prob.n_vir[Y]))
                for X, Y in ordered]
    sizes = [int(np.prod(s)) for s in shapes_T + shapes_U]
    offs = np.concatenate([[0], np.cumsum(sizes)])
    n = int(offs[-1])

    def unpack(x):
        T = [x[offs[k]:offs[k + 1]].reshape(shapes_T[k]) for k in range(cl.N)]
        tau = {xy: x[offs[cl.N + k]:offs[cl.N + k + 1]].reshape(shapes_U[k]) for k, xy in enumerate(ordered)}
        return T, tau

    def residual_rhs(x, with_source):
        """eps * unknown - (coupling terms of the unknowns) [- source]."""
        T, tau = unpack(x)
        out = np.zeros(n)
        for X in range(cl.N):
            O, V = cl.occ[X], cl.vir[X]
            r = np.zeros(shapes_T[X])
            for i in O:
                for i1 in O:
                    for a in V:
                        for a1 in V:
                            eps = cl.e(i) + cl.e(i1) - cl.e(a) - cl.e(a1)
                            c = intramonomer(cl, X, T, i, i1, a, a1) + _brute.pair_term(cl, X, tau, i, i1, a, a1)
                            src = cl.v(a, a1, i, i1) if with_source else 0.0
                            r[i.idx, i1.idx, a.idx, a1.idx] = eps * T[X][i.idx, i1.idx, a.idx, a1.idx] - c - src
            out[offs[X]:offs[X + 1]] = r.ravel()
        for k, (X, Y) in enumerate(ordered):
            u = _brute.brute_tau(cl, X, Y, T) if with_source else _tau_homog(cl, X, Y, T)
            eps = np.zeros(shapes_U[k])
            for i in cl.occ[X]:
                for a in cl.vir[X]:
                    for j in cl.occ[Y]:
                        for b in cl.vir[Y]:
                            eps[i.idx, a.idx, j.idx, b.idx] = cl.e(i) + cl.e(j) - cl.e(a) - cl.e(b)
            # brute_tau returns (source + couplings) / eps; eps * Tau - (source + couplings)
            out[offs[cl.N + k]:offs[cl.N + k + 1]] = (eps * tau[(X, Y)] - eps * u).ravel()
        return out

    b = -residual_rhs(np.zeros(n), True)
    A = np.zeros((n, n))
    for c in range(n):
        e = np.zeros(n)
        e[c] = 1.0
        A[:, c] = residual_rhs(e, False)
    x = np.linalg.solve(A, b)
    T, tau = unpack(x)
    e_m2, e_d2 = _brute.brute_energies(cl, T, tau)
    return T, tau, e_m2, e_d2


def _tau_homog(cl, X, Y, T):
    """Eq. 59's coupling terms alone (no source), divided by eps: brute_tau of
    the same T minus brute_tau of zero amplitudes."""
    zeros = [np.zeros_like(t) for t in T]
    return _brute.brute_tau(cl, X, Y, T) - _brute.brute_tau(cl, X, Y, zeros)
