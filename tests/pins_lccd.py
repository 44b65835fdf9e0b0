"""Pins of the full-monomer-equation oracle (oracle.mcpt_lccd) to facts outside itself.

Each pin takes the oracle module and returns (ok, detail); test_lccd_pins.py
runs them on the real oracle and test_lccd_mutations.py on broken copies, where
at least one pin must fail for every planted mistake.
"""
from __future__ import annotations

import itertools

import numpy as np

from synth import LccdIntegrals, concat_lccd, concat_problems, cubic_sites, lccd_integrals, make_lattice_problem
from . import _brute_lccd
from .pins import TEST_WORKLOAD, _rel, _safe

GROUP8 = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
          (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]


def tiny_lccd(sizes=((2, 3), (2, 2), (1, 3)), scale=3.0, cluster=0, sigma=0.03, general=False, seed=5):
    """A small cluster (all pairs) with its intramonomer integrals.  general:
    W, Q, J replaced by seeded normals with no permutational symmetry and K by
    normals with only the exact electron-exchange symmetry K[i,j,a,b] =
    K[j,i,b,a] (the ring integrals v^{ak}_{ic} and v^{ka}_{ci} are the same
    number by it, and both are read from K)."""
    sites = cubic_sites(len(sizes), 1, 1)
    p = make_lattice_problem(sites, None, sizes=list(sizes), workload=TEST_WORKLOAD, cluster=cluster,
                             coupling_scale=scale, k_scale=0.4)
    ints = lccd_integrals(p, sigma=sigma)
    if general:
        rng = np.random.default_rng(seed)
        for x in range(p.n_mono):
            g = rng.normal(0.0, 0.02, size=p.k_of(x).shape)
            p.k[p.k_off[x]:p.k_off[x + 1]] = (g + g.transpose(1, 0, 3, 2)).ravel()
        ints.w[:] = rng.normal(0.0, sigma, size=ints.w.shape)
        ints.q[:] = rng.normal(0.0, sigma, size=ints.q.shape)
        ints.j[:] = rng.normal(0.0, sigma, size=ints.j.shape)
    return p, ints


def physical_monomer(o, v, seed, sigma=0.06):
    """One monomer whose K, J, W, Q are all cut from one real two-electron
    tensor (pr|qs) with the full eightfold permutational symmetry."""
    rng = np.random.default_rng(seed)
    nmo = o + v
    g = rng.normal(0.0, sigma, size=(nmo,) * 4)
    g = sum(g.transpose(p) for p in GROUP8) / 8.0
    e = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, o)), np.sort(rng.uniform(0.2, 3.0, v))])
    O, V = slice(0, o), slice(o, nmo)
    p = make_lattice_problem(cubic_sites(1, 1, 1), None, sizes=[(o, v)], workload=TEST_WORKLOAD)
    p.eps[:] = e
    p.k[:] = g[V, O, V, O].transpose(1, 3, 0, 2).ravel()          # <ab|ij> = (ai|bj)
    ints = LccdIntegrals(p.n_occ.copy(), p.n_vir.copy(),
                         g[V, V, V, V].transpose(0, 2, 1, 3).ravel().copy(),   # <ab|cd> = (ac|bd)
                         g[O, O, O, O].transpose(0, 2, 1, 3).ravel().copy(),   # <ij|kl> = (ik|jl)
                         g[O, O, V, V].ravel().copy())                        # <ia|jb> = (ij|ab)
    return p, ints, g, e


def spin_orbital_lccd(g, e, o, v):
    """Textbook spin-orbital LCCD (Shavitt & Bartlett, ch. 9, linear terms of CCD):

        D_ij^ab t_ij^ab = <ab||ij> + 1/2 <ab||cd> t_ij^cd + 1/2 <kl||ij> t_kl^ab
                          + P(ij) P(ab) <kb||cj> t_ik^ac,     E = 1/4 <ij||ab> t_ij^ab

    with D = e_i + e_j - e_a - e_b, solved densely.  Returns (E, t in spin
    orbitals, spin-orbital index lists of the occupied and virtual orbitals)."""
    nmo = o + v
    occ = [(i, s) for i in range(o) for s in (0, 1)]
    vir = [(a, s) for a in range(o, nmo) for s in (0, 1)]
    so = occ + vir
    ns = len(so)
    A = np.zeros((ns,) * 4)
    for P, Q, R, S in itertools.product(range(ns), repeat=4):
        (p, sp), (q, sq), (r, sr), (s, ss) = so[P], so[Q], so[R], so[S]
        val = 0.0
        if sp == sr and sq == ss:
            val += g[p, r, q, s]
        if sp == ss and sq == sr:
            val -= g[p, s, q, r]
        A[P, Q, R, S] = val
    no = len(occ)
    oo, vv = slice(0, no), slice(no, ns)
    es = np.array([e[p] for p, _ in so])
    D = es[oo][:, None, None, None] + es[oo][None, :, None, None] - es[vv][None, None, :, None] \
        - es[vv][None, None, None, :]

    def lhs(t):
        r = D * t - 0.5 * np.einsum("abcd,ijcd->ijab", A[vv, vv, vv, vv], t)
        r -= 0.5 * np.einsum("klij,klab->ijab", A[oo, oo, oo, oo], t)
        x = np.einsum("kbcj,ikac->ijab", A[oo, vv, vv, oo], t)
        r -= x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
        return r

    shape = D.shape
    n = D.size
    M = np.zeros((n, n))
    for c in range(n):
        u = np.zeros(n)
        u[c] = 1.0
        M[:, c] = lhs(u.reshape(shape)).ravel()
    t = np.linalg.solve(M, A[vv, vv, oo, oo].transpose(2, 3, 0, 1).ravel()).reshape(shape)
    E = 0.25 * float(np.einsum("ijab,ijab->", A[oo, oo, vv, vv], t))
    return E, t, occ, vir


@_safe
def pin_spin_orbital_lccd(orc):
    """Physical integrals of one monomer: the isolated-monomer energy of step 5
    equals the spin-orbital LCCD energy, and T^{ab}_{ij} equals the alpha-beta
    spin-orbital amplitude t_{i alpha j beta}^{a alpha b beta}."""
    worst = 0.0
    for (o, v, seed) in [(2, 3, 11), (3, 2, 12), (2, 2, 13)]:
        p, ints, g, e = physical_monomer(o, v, seed)
        e_iso, T, status, _ = orc.isolated_lccd(p, ints, tol=1e-15, max_sweeps=400)
        if status != 0:
            return False, f"isolated LCCD status {status}"
        E, t, occ, vir = spin_orbital_lccd(g, e, o, v)
        ia = [occ.index((i, 0)) for i in range(o)]
        jb = [occ.index((i, 1)) for i in range(o)]
        aa = [vir.index((a, 0)) for a in range(o, o + v)]
        bb = [vir.index((a, 1)) for a in range(o, o + v)]
        worst = max(worst, abs(e_iso[0] - E) / abs(E), _rel(T[0], t[np.ix_(ia, jb, aa, bb)]))
    return worst < 1e-11, f"worst relative difference {worst:.3e}"


@_safe
def pin_no_pairs_equals_isolated(orc):
    """Without pairs, step 6 is step 5: E_M2(X) equals E_LCCD(X) and dE_M2 = 0."""
    p, ints = tiny_lccd()
    q = p.subset_pairs(np.zeros(p.n_pair, dtype=bool))
    r = orc.solve(q, ints, tol=1e-14)
    worst = _rel(r.e_m2, r.e_m2_0)
    return r.status == 0 and worst < 1e-13, f"status {r.status}, worst {worst:.3e}"


@_safe
def pin_brute_force_lccd(orc):
    """Fixed sweep counts (isolated and coupled) agree element by element with
    the brute-force twin (generic integral lookup, terms looped as printed),
    for physical-symmetry and for general integrals."""
    worst = 0.0
    for general, k in [(False, 0), (False, 1), (False, 2), (True, 2)]:
        p, ints = tiny_lccd(general=general)
        r = orc.solve(p, ints, tol=0.0, max_sweeps=k)
        T, tau, e_m2, e_d2, e_iso = _brute_lccd.brute_lccd_sweeps(p, ints, k, k)
        for x in range(p.n_mono):
            worst = max(worst, _rel(r.T[x], T[x]))
        for q in range(p.n_pair):
            x, y = (int(t) for t in p.pairs[q])
            worst = max(worst, _rel(r.Tau[q], tau[(x, y)]))
            worst = max(worst, abs(r.e_d2[q] - e_d2[(x, y)]) / abs(e_d2[(x, y)]))
        worst = max(worst, _rel(r.e_m2, e_m2), _rel(r.e_m2_0, e_iso))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_dense_lccd(orc):
    """The converged coupled iteration equals the LAPACK solution of the stacked
    linear system of Eqs. 58-59 (all printed terms of Eq. 58)."""
    worst = 0.0
    for general in (False, True):
        p, ints = tiny_lccd(sizes=((2, 3), (1, 3), (2, 2)), general=general)
        r = orc.solve(p, ints, tol=1e-15, max_sweeps=400)
        if r.status != 0:
            return False, f"status {r.status}"
        T, tau, e_m2, e_d2 = _brute_lccd.dense_lccd(p, ints)
        for x in range(p.n_mono):
            worst = max(worst, _rel(r.T[x], T[x]))
        for q in range(p.n_pair):
            x, y = (int(t) for t in p.pairs[q])
            worst = max(worst, _rel(r.Tau[q], tau[(x, y)]))
        worst = max(worst, _rel(r.e_m2, e_m2))
    return worst < 1e-10, f"worst relative difference {worst:.3e}"


@_safe
def pin_lccd_scaling_bitwise(orc):
    """(eps, K, J, W, Q, V) -> 8 x: T unchanged and every energy times 8, bitwise."""
    p, ints = tiny_lccd()
    q, qi = tiny_lccd()
    for a in (q.eps, q.k, q.v, qi.w, qi.q, qi.j):
        a *= 8.0
    r0 = orc.solve(p, ints, tol=0.0, max_sweeps=3)
    r1 = orc.solve(q, qi, tol=0.0, max_sweeps=3)
    ok = all(np.array_equal(a, b) for a, b in zip(r0.T, r1.T))
    ok &= np.array_equal(8.0 * r0.e_m2, r1.e_m2) and np.array_equal(8.0 * r0.e_d2, r1.e_d2)
    ok &= np.array_equal(8.0 * r0.e_m2_0, r1.e_m2_0)
    return bool(ok), "bitwise" if ok else "differs"


@_safe
def pin_lccd_relabel(orc):
    """Relabelling monomers and storing pairs reversed permutes the per-monomer
    results and leaves the energies unchanged."""
    p, ints = tiny_lccd(sizes=((2, 3), (1, 4), (3, 2), (2, 2)))
    perm = np.array([2, 0, 3, 1])
    flip = np.arange(p.n_pair) % 2 == 0
    q = p.relabel(perm, flip)
    qi = ints.subset(perm)
    r0 = orc.solve(p, ints, tol=1e-14)
    r1 = orc.solve(q, qi, tol=1e-14)
    worst = abs(r0.e_total - r1.e_total) / abs(r0.e_total)
    worst = max(worst, _rel(r1.e_m2, r0.e_m2[perm]), _rel(r1.e_m2_0, r0.e_m2_0[perm]), _rel(r1.e_d2, r0.e_d2))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_lccd_orbital_permutation(orc):
    """Reordering the occupied and virtual orbitals of one monomer consistently in
    eps, K, J, W, Q and V leaves every energy unchanged."""
    p, ints = tiny_lccd(sizes=((2, 3), (3, 2)))
    q, qi = tiny_lccd(sizes=((2, 3), (3, 2)))
    x = 0
    o, v = int(p.n_occ[x]), int(p.n_vir[x])
    po, pv = np.array([1, 0]), np.array([2, 0, 1])
    eo, ev = p.eps_of(x)
    q.eps[q.eps_off[x]:q.eps_off[x] + o] = eo[po]
    q.eps[q.eps_off[x] + o:q.eps_off[x + 1]] = ev[pv]
    q.k[q.k_off[x]:q.k_off[x + 1]] = p.k_of(x)[np.ix_(po, po, pv, pv)].ravel()
    qi.w[qi.w_off[x]:qi.w_off[x + 1]] = ints.w_of(x)[np.ix_(pv, pv, pv, pv)].ravel()
    qi.q[qi.q_off[x]:qi.q_off[x + 1]] = ints.q_of(x)[np.ix_(po, po, po, po)].ravel()
    qi.j[qi.j_off[x]:qi.j_off[x + 1]] = ints.j_of(x)[np.ix_(po, po, pv, pv)].ravel()
    for k in range(p.n_pair):
        X, Y = (int(t) for t in p.pairs[k])
        V = p.v_of(k)
        if X == x:
            V = V[np.ix_(po, pv, np.arange(V.shape[2]), np.arange(V.shape[3]))]
        elif Y == x:
            V = V[np.ix_(np.arange(V.shape[0]), np.arange(V.shape[1]), po, pv)]
        q.v[q.v_off[k]:q.v_off[k + 1]] = V.ravel()
    r0 = orc.solve(p, ints, tol=1e-15)
    r1 = orc.solve(q, qi, tol=1e-15)
    worst = max(_rel(r1.e_m2, r0.e_m2), _rel(r1.e_d2, r0.e_d2), _rel(r1.e_m2_0, r0.e_m2_0))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_lccd_disconnected(orc):
    """Two clusters with no pairs between them: the union's energies are those
    of the separate solves."""
    a, ia = tiny_lccd(cluster=1)
    b, ib = tiny_lccd(sizes=((1, 3), (2, 2)), cluster=2)
    u = concat_problems([a, b])
    iu = concat_lccd([ia, ib])
    ra, rb, ru = orc.solve(a, ia, tol=1e-15), orc.solve(b, ib, tol=1e-15), orc.solve(u, iu, tol=1e-15)
    worst = max(_rel(ru.e_m2, np.concatenate([ra.e_m2, rb.e_m2])),
                _rel(ru.e_d2, np.concatenate([ra.e_d2, rb.e_d2])),
                _rel(ru.e_m2_0, np.concatenate([ra.e_m2_0, rb.e_m2_0])))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


ALL_LCCD_PINS = [
    pin_spin_orbital_lccd, pin_no_pairs_equals_isolated, pin_brute_force_lccd, pin_dense_lccd,
    pin_lccd_scaling_bitwise, pin_lccd_relabel, pin_lccd_orbital_permutation, pin_lccd_disconnected,
]
