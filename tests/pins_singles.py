"""Pins of the singles oracle to facts outside itself.

Each pin takes the singles oracle module and returns (ok, detail); the suite
runs against the real module in test_singles_pins.py and against broken copies
in test_singles_mutations.py, where every planted mistake must fail a pin.
"""
from __future__ import annotations

import numpy as np

from synth import concat_problems, cubic_sites, make_lattice_problem, singles_source
from . import _brute
from .pins import TEST_WORKLOAD, _rel, _safe, tiny


def _w_blocks(p, w):
    out, off = [], 0
    for x in range(p.n_mono):
        o, v = int(p.n_occ[x]), int(p.n_vir[x])
        out.append(np.asarray(w[off:off + o * v]).reshape(o, v))
        off += o * v
    return out


def _tiny_singles(scale=1.5, sizes=((2, 3), (2, 4), (3, 2), (1, 3))):
    sites = cubic_sites(len(sizes), 1, 1)
    p = make_lattice_problem(sites, None, sizes=list(sizes), workload=TEST_WORKLOAD, coupling_scale=scale)
    return p, singles_source(p)


@_safe
def pin_singles_zero_coupling(ms):
    """No pairs: one sweep, and each monomer's energy is the textbook
    second-order singles energy 2 sum |w_ia|^2 / (e_i - e_a)."""
    p, w = _tiny_singles()
    p = p.subset_pairs(np.zeros(p.n_pair, dtype=bool))
    r = ms.solve(p, w, tol=1e-14, max_sweeps=5)
    wb = _w_blocks(p, w)
    ref = []
    for x in range(p.n_mono):
        eo, ev = p.eps_of(x)
        s = 0.0
        for i in range(len(eo)):
            for a in range(len(ev)):
                s += 2.0 * wb[x][i, a] ** 2 / (eo[i] - ev[a])
        ref.append(s)
    ok = r.status == 0 and r.sweeps == 1 and _rel(r.e_m1, ref) < 1e-13 and all(e < 0 for e in r.e_m1)
    return ok, f"status {r.status} sweeps {r.sweeps} rel {_rel(r.e_m1, ref):.2e}"


@_safe
def pin_singles_brute_force_sweeps(ms):
    """Three fixed sweeps against pure-Python loops that place every index of
    Eq. (57) through a generic <pq|rs> lookup."""
    p, w = _tiny_singles()
    cl = _brute.Cluster(p)
    wb = _w_blocks(p, w)
    t = _brute.brute_singles_first_order(cl, wb)
    for _ in range(3):
        t = _brute.brute_singles_sweep(cl, wb, t)
    e = _brute.brute_singles_energy(cl, wb, t)
    r = ms.solve(p, w, tol=0.0, max_sweeps=3)
    err_t = max(_rel(r.t[x], t[x]) for x in range(p.n_mono))
    return r.sweeps == 3 and err_t < 1e-12 and _rel(r.e_m1, e) < 1e-12, f"t {err_t:.2e} e {_rel(r.e_m1, e):.2e}"


@_safe
def pin_singles_dense_solve(ms):
    """The converged amplitudes solve spin-orbital linear singles,
        (e_i - e_a) t_i^a = w_i^a + sum over spin orbitals k, c of the neighbour
                            monomers of <ak||ic> t_k^c,
    assembled over every spin orbital of the cluster (integrals through the
    generic <pq|rs> lookup; the exchange part vanishes between monomers) and
    solved by a dense LAPACK solve; the closed-shell alpha and beta amplitudes
    come out equal and equal the oracle's.  Fixes the spin sum of the pair term
    of Eq. 57 (twice the printed term)."""
    p, w = _tiny_singles(scale=1.2, sizes=((2, 3), (3, 2), (2, 2), (1, 4), (2, 1)))
    cl = _brute.Cluster(p)
    wb = _w_blocks(p, w)
    so = [(X, i, a, s) for X in range(p.n_mono) for i in cl.occ[X] for a in cl.vir[X] for s in _brute.SPINS]
    n = len(so)
    A = np.zeros((n, n))
    rhs = np.zeros(n)
    for r_, (X, i, a, s) in enumerate(so):
        A[r_, r_] = cl.e(i) - cl.e(a)
        rhs[r_] = wb[X][i.idx, a.idx]
        for c_, (Y, k, c, sk) in enumerate(so):
            if Y not in cl.neighbours[X]:
                continue
            # <ak||ic> = <ak|ic> - <ak|ci> over spin orbitals
            A[r_, c_] -= _brute.v_spin(cl, a, s, k, sk, i, s, c, sk) - _brute.v_spin(cl, a, s, k, sk, c, sk, i, s)
    t_so = np.linalg.solve(A, rhs)
    t_a = np.array([t_so[r_] for r_, q in enumerate(so) if q[3] == 0])
    t_b = np.array([t_so[r_] for r_, q in enumerate(so) if q[3] == 1])
    r = ms.solve(p, w, tol=1e-14, max_sweeps=2000)
    t = np.concatenate([tx.ravel() for tx in r.t])
    e_ref = 2.0 * float(np.asarray(w) @ t_a)
    ok = r.status == 0 and _rel(t_b, t_a) < 1e-13 and _rel(t, t_a) < 1e-10 and \
        abs(r.e_total - e_ref) < 1e-10 * abs(e_ref)
    return ok, f"status {r.status} sweeps {r.sweeps} t {_rel(t, t_a):.2e} E {r.e_total} vs {e_ref}"


@_safe
def pin_singles_relabel_and_orientation(ms):
    """Renumbering monomers and storing pairs reversed permutes the energies
    and changes nothing else."""
    p, w = _tiny_singles()
    perm = [2, 0, 3, 1]
    flip = np.arange(p.n_pair) % 2 == 0
    q = p.relabel(perm, flip)
    wb = _w_blocks(p, w)
    wq = np.concatenate([wb[x].ravel() for x in perm])
    a = ms.solve(p, w, tol=1e-13)
    b = ms.solve(q, wq, tol=1e-13)
    return _rel(b.e_m1, a.e_m1[perm]) < 1e-12 and a.sweeps == b.sweeps, f"rel {_rel(b.e_m1, a.e_m1[perm]):.2e}"


@_safe
def pin_singles_disconnected_additivity(ms):
    """Two clusters with no pairs between them solve as if alone."""
    p1, w1 = _tiny_singles()
    sites = cubic_sites(2, 1, 1)
    p2 = make_lattice_problem(sites, None, sizes=[(2, 2), (3, 3)], workload=TEST_WORKLOAD, cluster=5,
                              coupling_scale=1.5)
    w2 = singles_source(p2)
    u = concat_problems([p1, p2])
    r = ms.solve(u, np.concatenate([w1, w2]), tol=1e-13)
    a = ms.solve(p1, w1, tol=1e-13)
    b = ms.solve(p2, w2, tol=1e-13)
    ref = np.concatenate([a.e_m1, b.e_m1])
    return _rel(r.e_m1, ref) < 1e-12, f"rel {_rel(r.e_m1, ref):.2e}"


@_safe
def pin_singles_intramonomer_spin_orbital(ms):
    """With the intramonomer classes: on a dimer whose integrals are all cut from
    one real two-electron tensor g (no exchange between the monomers), the
    converged amplitudes equal spin-orbital linear singles,
        (e_i - e_a) t_i^a = w_i^a + sum over every occupied k and virtual c spin
                            orbital of the dimer of <ak||ic> t_k^c,
    with <ak|ic> = (ai|kc) = g[a, i, k, c] and <ak|ci> = g[a, c, k, i] read from g
    itself, solved densely; alpha and beta amplitudes come out equal.  Fixes the
    2v - v combination of Eq. 57's intramonomer term, its integral classes and
    the spin sum of the pair term together."""
    from .pins_dimer import physical_dimer
    worst = 0.0
    for sx, sy, seed in [((2, 3), (1, 3), 41), ((2, 2), (3, 2), 42)]:
        p, ints, _, g, e, orbs = physical_dimer(sx, sy, seed)
        rng = np.random.default_rng(seed)
        w = rng.normal(0.0, 0.05, size=sum(p.n_ov(x) for x in range(p.n_mono)))
        occ = [k for k, (_, o, _) in enumerate(orbs) if o]
        vir = [k for k, (_, o, _) in enumerate(orbs) if not o]
        so = [(m, i, a, s_) for m in (0, 1) for i in occ if orbs[i][0] == m
              for a in vir if orbs[a][0] == m for s_ in (0, 1)]
        n = len(so)
        A = np.zeros((n, n))
        rhs = np.zeros(n)
        woff = {0: 0, 1: p.n_ov(0)}
        for r_, (m, i, a, s_) in enumerate(so):
            A[r_, r_] = e[i] - e[a]
            rhs[r_] = w[woff[m] + orbs[i][2] * int(p.n_vir[m]) + orbs[a][2]]
            for c_, (m2, k, c, sk) in enumerate(so):
                direct = g[a, i, k, c]                         # <ak|ic>, spins of (a,i) and (k,c) each kept
                exch = g[a, c, k, i] if sk == s_ else 0.0      # <ak|ci> needs a, c and k, i of one spin
                A[r_, c_] -= direct - exch
        t_so = np.linalg.solve(A, rhs)
        t_a = np.array([t_so[r_] for r_, q in enumerate(so) if q[3] == 0])
        t_b = np.array([t_so[r_] for r_, q in enumerate(so) if q[3] == 1])
        r = ms.solve(p, w, tol=1e-14, max_sweeps=3000, ints=ints)
        if r.status != 0:
            return False, f"status {r.status}"
        t = np.concatenate([tx.ravel() for tx in r.t])
        worst = max(worst, _rel(t_b, t_a), _rel(t, t_a))
    return worst < 1e-10, f"worst relative difference {worst:.3e}"


@_safe
def pin_singles_divergence_detected(ms):
    """A coupling far above the denominators makes the iteration diverge, and
    the rule says so."""
    p, w = _tiny_singles(scale=400.0)
    r = ms.solve(p, w, tol=1e-10, max_sweeps=200)
    return r.status == -5, f"status {r.status} sweeps {r.sweeps}"


ALL_SINGLES_PINS = [
    pin_singles_zero_coupling,
    pin_singles_brute_force_sweeps,
    pin_singles_dense_solve,
    pin_singles_relabel_and_orientation,
    pin_singles_disconnected_additivity,
    pin_singles_divergence_detected,
    pin_singles_intramonomer_spin_orbital,
]
