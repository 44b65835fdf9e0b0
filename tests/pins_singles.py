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
    """The converged amplitudes solve the assembled linear system
    (diag(e_i - e_a) - A) t = w, A holding V_XY and V_XY^T blocks, by a dense
    LAPACK solve."""
    p, w = _tiny_singles(scale=2.0, sizes=((2, 3), (3, 2), (2, 2), (1, 4), (2, 1)))
    n = [p.n_ov(x) for x in range(p.n_mono)]
    off = np.concatenate([[0], np.cumsum(n)])
    A = np.zeros((off[-1], off[-1]))
    for q in range(p.n_pair):
        x, y = (int(t) for t in p.pairs[q])
        B = np.asarray(p.v_of(q)).reshape(n[x], n[y])
        A[off[x]:off[x + 1], off[y]:off[y + 1]] = B
        A[off[y]:off[y + 1], off[x]:off[x + 1]] = B.T
    d = np.concatenate([(p.eps_of(x)[0][:, None] - p.eps_of(x)[1][None, :]).ravel() for x in range(p.n_mono)])
    t_ref = np.linalg.solve(np.diag(d) - A, w)
    r = ms.solve(p, w, tol=1e-14, max_sweeps=2000)
    t = np.concatenate([tx.ravel() for tx in r.t])
    e_ref = 2.0 * float(w @ t_ref)
    ok = r.status == 0 and _rel(t, t_ref) < 1e-10 and abs(r.e_total - e_ref) < 1e-10 * abs(e_ref)
    return ok, f"status {r.status} sweeps {r.sweeps} t {_rel(t, t_ref):.2e} E {r.e_total} vs {e_ref}"


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
]
