"""Pins of the dimer-internal oracle (oracle.mcpt_dimer) to facts outside itself.

Each pin takes the oracle module and returns (ok, detail); test_dimer_pins.py
runs them on the real oracle and test_dimer_mutations.py on broken copies,
where at least one pin must fail for every planted mistake.
"""
from __future__ import annotations

import itertools

import numpy as np

from synth import DimerIntegrals, LccdIntegrals, cubic_sites, dimer_integrals, lccd_integrals, make_lattice_problem
from .pins import TEST_WORKLOAD, _rel, _safe
from .pins_lccd import GROUP8

GROUP4 = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2)]


def physical_dimer(sx, sy, seed, sigma=0.05, sigma_xy=0.04):
    """Two monomers whose every integral is cut from one real two-electron tensor
    (pq|rs) of the dimer's orbitals with no exchange between the monomers: (pq|rs)
    is nonzero only when p, q sit on one monomer and r, s on one monomer.
    Returns (problem, intramonomer integrals, dimer integrals, g, orbital energies,
    orbital table [(monomer, occupied?, local index)])."""
    rng = np.random.default_rng(seed)
    (ox, vx), (oy, vy) = sx, sy
    nx, ny = ox + vx, oy + vy
    sym = lambda a, grp: sum(a.transpose(p) for p in grp) / len(grp)
    gx = sym(rng.normal(0.0, sigma, size=(nx,) * 4), GROUP8)
    gy = sym(rng.normal(0.0, sigma, size=(ny,) * 4), GROUP8)
    gxy = sym(rng.normal(0.0, sigma_xy, size=(nx, nx, ny, ny)), GROUP4)
    n = nx + ny
    g = np.zeros((n,) * 4)
    X, Y = slice(0, nx), slice(nx, n)
    g[X, X, X, X] = gx
    g[Y, Y, Y, Y] = gy
    g[X, X, Y, Y] = gxy
    g[Y, Y, X, X] = gxy.transpose(2, 3, 0, 1)
    ex = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, ox)), np.sort(rng.uniform(0.2, 3.0, vx))])
    ey = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, oy)), np.sort(rng.uniform(0.2, 3.0, vy))])
    orbs = [(0, k < ox, k if k < ox else k - ox) for k in range(nx)] + \
           [(1, k < oy, k if k < oy else k - oy) for k in range(ny)]

    p = make_lattice_problem(cubic_sites(2, 1, 1), None, sizes=[sx, sy], workload=TEST_WORKLOAD)
    assert p.n_pair == 1 and tuple(p.pairs[0]) == (0, 1)
    p.eps[:] = np.concatenate([ex, ey])
    OX, VX, OY, VY = slice(0, ox), slice(ox, nx), slice(0, oy), slice(oy, ny)
    p.k[:] = np.concatenate([gx[VX, OX, VX, OX].transpose(1, 3, 0, 2).ravel(),      # K[i,j,a,b] = (ai|bj)
                             gy[VY, OY, VY, OY].transpose(1, 3, 0, 2).ravel()])
    p.v[:] = gxy[VX, OX, VY, OY].transpose(1, 0, 3, 2).ravel()                    # V[i,a,j,b] = (ai|bj)
    ints = LccdIntegrals(p.n_occ.copy(), p.n_vir.copy(),
                         np.concatenate([gx[VX, VX, VX, VX].transpose(0, 2, 1, 3).ravel(),
                                         gy[VY, VY, VY, VY].transpose(0, 2, 1, 3).ravel()]),
                         np.concatenate([gx[OX, OX, OX, OX].transpose(0, 2, 1, 3).ravel(),
                                         gy[OY, OY, OY, OY].transpose(0, 2, 1, 3).ravel()]),
                         np.concatenate([gx[OX, OX, VX, VX].ravel(), gy[OY, OY, VY, VY].ravel()]))
    dints = DimerIntegrals(np.array([[ox, vx, oy, vy]], dtype=np.int64),
                           gxy[VX, VX, VY, VY].transpose(0, 2, 1, 3).ravel().copy(),   # (a a1|b b1) -> [a,b,a1,b1]
                           gxy[OX, OX, OY, OY].transpose(0, 2, 1, 3).ravel().copy(),   # (i1 i|j1 j) -> [i1,j1,i,j]
                           gxy[OX, OX, VY, VY].ravel().copy(),                         # (i1 i|b b1)
                           gxy[VX, VX, OY, OY].transpose(2, 3, 0, 1).ravel().copy())   # (j1 j|a a1)
    return p, ints, dints, g, np.concatenate([ex, ey]), orbs


def restricted_lccd(g, e, orbs):
    """Textbook spin-orbital LCCD (Shavitt & Bartlett, ch. 9):

        D_ij^ab t_ij^ab = <ab||ij> + 1/2 <ab||cd> t_ij^cd + 1/2 <kl||ij> t_kl^ab
                          + P(ij) P(ab) <kb||cj> t_ik^ac,     E = 1/4 <ij||ab> t_ij^ab

    solved densely in the space of the double excitations that keep each
    electron on its monomer (i -> a and j -> b, or i -> b and j -> a, within one
    monomer each).  Returns (E, t, spin-orbital lists of occupied and virtual
    orbitals as (spatial index, spin))."""
    occ = [(k, s) for k, (_, o, _) in enumerate(orbs) if o for s in (0, 1)]
    vir = [(k, s) for k, (_, o, _) in enumerate(orbs) if not o for s in (0, 1)]
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
    mon = np.array([orbs[p][0] for p, _ in so])
    mi, mv = mon[:no], mon[no:]
    keep = ((mi[:, None, None, None] == mv[None, None, :, None]) & (mi[None, :, None, None] == mv[None, None, None, :])) | \
           ((mi[:, None, None, None] == mv[None, None, None, :]) & (mi[None, :, None, None] == mv[None, None, :, None]))
    es = np.array([e[p] for p, _ in so])
    D = es[oo][:, None, None, None] + es[oo][None, :, None, None] - es[vv][None, None, :, None] \
        - es[vv][None, None, None, :]

    def lhs(t):
        r = D * t - 0.5 * np.einsum("abcd,ijcd->ijab", A[vv, vv, vv, vv], t)
        r -= 0.5 * np.einsum("klij,klab->ijab", A[oo, oo, oo, oo], t)
        x = np.einsum("kbcj,ikac->ijab", A[oo, vv, vv, oo], t)
        r -= x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
        return r

    idx = np.flatnonzero(keep.ravel())
    M = np.zeros((idx.size, idx.size))
    for c, flat in enumerate(idx):
        u = np.zeros(D.size)
        u[flat] = 1.0
        M[:, c] = lhs(u.reshape(D.shape)).ravel()[idx]
    src = A[vv, vv, oo, oo].transpose(2, 3, 0, 1).ravel()[idx]
    t = np.zeros(D.size)
    t[idx] = np.linalg.solve(M, src)
    t = t.reshape(D.shape)
    E = 0.25 * float(np.einsum("ijab,ijab->", A[oo, oo, vv, vv], t))
    return E, t, occ, vir


def compare_restricted_lccd(r, sx, sy, g, e, orbs) -> float:
    """Worst relative difference between an oracle result r on a two-monomer
    problem and restricted spin-orbital LCCD on the same integrals: energy
    E_M2(X) + E_M2(Y) + E_D2(XY), T_X and T_Y against the alpha-beta amplitudes of
    each monomer, Tau^{ab}_{ij} against t_{i alpha j beta}^{a alpha b beta}."""
    E, t, occ, vir = restricted_lccd(g, e, orbs)
    e_mcpt = float(np.sum(r.e_m2) + np.sum(r.e_d2))
    worst = abs(e_mcpt - E) / abs(E)
    loc = lambda m, o_flag, k, s, lst: lst.index((next(q for q, ob in enumerate(orbs)
                                                      if ob == (m, o_flag, k)), s))
    (ox, vx), (oy, vy) = sx, sy
    for m, (o, v) in enumerate((sx, sy)):
        ii = [loc(m, True, k, 0, occ) for k in range(o)]
        jj = [loc(m, True, k, 1, occ) for k in range(o)]
        aa = [loc(m, False, k, 0, vir) for k in range(v)]
        bb = [loc(m, False, k, 1, vir) for k in range(v)]
        ref = t[np.ix_(ii, jj, aa, bb)]
        if np.any(ref):
            worst = max(worst, _rel(r.T[m], ref))
        else:
            worst = max(worst, float(np.max(np.abs(r.T[m]))))
    ii = [loc(0, True, k, 0, occ) for k in range(ox)]
    aa = [loc(0, False, k, 0, vir) for k in range(vx)]
    jj = [loc(1, True, k, 1, occ) for k in range(oy)]
    bb = [loc(1, False, k, 1, vir) for k in range(vy)]
    return max(worst, _rel(r.Tau[0], t[np.ix_(ii, jj, aa, bb)].transpose(0, 2, 1, 3)))


@_safe
def pin_restricted_lccd(orc):
    """Physical dimer integrals without exchange between the monomers: the
    converged E_M2(X) + E_M2(Y) + E_D2(XY) equals the restricted spin-orbital
    LCCD energy, T_X and T_Y equal the alpha-beta amplitudes of each monomer and
    Tau^{ab}_{ij} equals t_{i alpha j beta}^{a alpha b beta} (i, a on X; j, b on Y).
    This holds with the pair term of Eq. 58 summed over both spins of k, c on Y
    (the printed term is half of it), and with every dimer-internal term as
    printed."""
    worst = 0.0
    for sx, sy, seed in [((1, 2), (1, 2), 21), ((2, 2), (1, 3), 22), ((1, 3), (2, 2), 23)]:
        p, ints, dints, g, e, orbs = physical_dimer(sx, sy, seed)
        r = orc.solve(p, ints, dints, tol=1e-15, max_sweeps=400)
        if r.status != 0:
            return False, f"status {r.status}"
        worst = max(worst, compare_restricted_lccd(r, sx, sy, g, e, orbs))
    return worst < 1e-10, f"worst relative difference {worst:.3e}"


def tiny_dimer(sizes=((2, 3), (2, 2), (1, 3)), scale=3.0, sigma=0.03, dsigma=0.03):
    sites = cubic_sites(len(sizes), 1, 1)
    p = make_lattice_problem(sites, None, sizes=list(sizes), workload=TEST_WORKLOAD, coupling_scale=scale,
                             k_scale=0.4)
    return p, lccd_integrals(p, sigma=sigma), dimer_integrals(p, sigma=dsigma)


def _reverse(p, ints, dints):
    """The same cluster with every stored pair reversed (Y first): V_YX = V_XY^T and
    the dimer classes relabelled to match."""
    q = make_lattice_problem(p.sites, None, sizes=[(int(a), int(b)) for a, b in zip(p.n_occ, p.n_vir)],
                             workload=TEST_WORKLOAD)
    q.eps[:] = p.eps
    q.k[:] = p.k
    q.pairs = np.ascontiguousarray(p.pairs[:, ::-1])
    vs, shapes, ws, qs, cxs, cys = [], [], [], [], [], []
    for k in range(p.n_pair):
        vs.append(np.ascontiguousarray(p.v_of(k).transpose(2, 3, 0, 1)).ravel())
        ox, vx, oy, vy = (int(t) for t in dints.shapes[k])
        shapes.append((oy, vy, ox, vx))
        ws.append(np.ascontiguousarray(dints.w_of(k).transpose(1, 0, 3, 2)).ravel())
        qs.append(np.ascontiguousarray(dints.q_of(k).transpose(1, 0, 3, 2)).ravel())
        cxs.append(dints.cy_of(k).ravel())
        cys.append(dints.cx_of(k).ravel())
    q.v = np.concatenate(vs)
    q.__post_init__()
    return q, ints, DimerIntegrals(np.array(shapes, dtype=np.int64), np.concatenate(ws), np.concatenate(qs),
                                   np.concatenate(cxs), np.concatenate(cys))


@_safe
def pin_pair_orientation(orc):
    """Storing every pair the other way round (Y first, every class relabelled)
    changes no energy and no amplitude: the equation of Eq. 59 names X and Y
    symmetrically."""
    p, ints, dints = tiny_dimer()
    a = orc.solve(p, ints, dints, tol=0, max_sweeps=6)
    q, ints2, d2 = _reverse(p, ints, dints)
    b = orc.solve(q, ints2, d2, tol=0, max_sweeps=6)
    worst = max(_rel(b.e_d2, a.e_d2), _rel(b.e_m2, a.e_m2),
                max(_rel(b.Tau[k], a.Tau[k].transpose(2, 3, 0, 1)) for k in range(p.n_pair)),
                max(_rel(b.T[x], a.T[x]) for x in range(p.n_mono)))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_zero_classes_single_sweep(orc):
    """Before the first sweep Tau is zero, so the first sweep's Tau is the reduced
    equation's and the dimer terms enter from the second sweep on: one sweep
    equals the full-monomer-equation oracle's sweep, two differ."""
    from oracle import mcpt_lccd
    p, ints, dints = tiny_dimer()
    a = orc.solve(p, ints, dints, tol=0, max_sweeps=1)
    b = mcpt_lccd.solve(p, ints, tol=0, max_sweeps=1)
    one = max(_rel(a.T[x], b.T[x]) for x in range(p.n_mono))
    a2 = orc.solve(p, ints, dints, tol=0, max_sweeps=2)
    b2 = mcpt_lccd.solve(p, ints, tol=0, max_sweeps=2)
    two = max(_rel(a2.T[x], b2.T[x]) for x in range(p.n_mono))
    return one < 1e-15 and two > 1e-6, f"one sweep {one:.3e}, two sweeps {two:.3e}"


ALL_PINS = [pin_restricted_lccd, pin_pair_orientation, pin_zero_classes_single_sweep]
