"""Pins of the oracle to facts outside itself.

Each pin takes the oracle module and returns (ok, detail).  The pin suite runs
against the real oracle in test_oracle_pins.py, and against deliberately
broken copies of it in test_oracle_mutations.py, where at least one pin must
fail for every planted mistake.
"""
from __future__ import annotations

import numpy as np

from synth import cubic_sites, make_lattice_problem, make_workload, concat_problems
from . import _brute

TEST_WORKLOAD = 900


def tiny(sizes=((2, 3), (2, 4), (3, 2)), scale=3.0, cutoff=None, workload=TEST_WORKLOAD, cluster=0):
    sites = cubic_sites(len(sizes), 1, 1)
    return make_lattice_problem(sites, cutoff, sizes=list(sizes), workload=workload,
                                cluster=cluster, coupling_scale=scale)


def general_k(p, seed=7):
    """Replace the intra blocks by seeded normals with no permutational symmetry
    (the equations do not assume any; this separates the occupied from the
    virtual index swap, which coincide on pair-symmetric amplitudes)."""
    rng = np.random.default_rng(seed)
    p.k[:] = rng.normal(0.0, 0.05, size=p.k.shape)
    return p


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return float(np.max(np.abs(a - b))) / den if a.size else 0.0


def _safe(fn):
    def wrapped(orc):
        try:
            return fn(orc)
        except Exception as exc:   # a broken oracle may also raise
            return False, f"raised {type(exc).__name__}: {exc}"
    wrapped.__name__ = fn.__name__
    return wrapped


@_safe
def pin_zero_coupling_mp2(orc):
    """No pairs: each monomer's energy is the textbook closed-shell second-order
    energy, reached in one sweep."""
    p = tiny().subset_pairs(np.zeros(3, dtype=bool))
    r = orc.solve(p, tol=1e-14, max_sweeps=5)
    ok = r.status == 0 and r.sweeps == 1
    for x in range(p.n_mono):
        px = make_lattice_problem(cubic_sites(1, 1, 1), None, sizes=[(int(p.n_occ[x]), int(p.n_vir[x]))],
                                  workload=TEST_WORKLOAD)
        px.k[:] = p.k_of(x).ravel()
        px.eps[:] = p.eps[p.eps_off[x]:p.eps_off[x + 1]]
        ref = _brute.supersystem_mp2(px)
        ok &= abs(r.e_m2[x] - ref) <= 1e-13 * abs(ref)
        ok &= abs(r.e_m2_0[x] - ref) <= 1e-13 * abs(ref)
    return ok, f"status={r.status} sweeps={r.sweeps} e_m2={r.e_m2}"


@_safe
def pin_dispersion_mp2(orc):
    """Intra blocks zero, zero sweeps: the dimer energies summed over unordered
    pairs equal the textbook closed-shell second-order energy of the cluster."""
    p = tiny()
    p.k[:] = 0.0
    r = orc.solve(p, tol=0.0, max_sweeps=0)
    ref = _brute.supersystem_mp2(p)
    ok = abs(r.e_total - ref) <= 1e-13 * abs(ref) and abs(r.e_mono) == 0.0
    return ok, f"oracle {r.e_total!r} textbook {ref!r}"


@_safe
def pin_brute_force_sweeps(orc):
    """Fixed sweep counts agree with the brute-force twin (ordered pairs,
    generic integral lookup) element by element."""
    worst = 0.0
    ok = True
    for p, k in [(tiny(), 0), (tiny(), 1), (tiny(), 2), (general_k(tiny()), 2)]:
        r = orc.solve(p, tol=0.0, max_sweeps=k)
        T, tau, e_m2, e_d2 = _brute.brute_sweeps(p, k)
        for x in range(p.n_mono):
            worst = max(worst, _rel(r.T[x], T[x]))
        for q in range(p.n_pair):
            x, y = (int(t) for t in p.pairs[q])
            worst = max(worst, _rel(r.Tau[q], tau[(x, y)]))
            worst = max(worst, _rel(r.Tau[q].transpose(2, 3, 0, 1), tau[(y, x)]))
            worst = max(worst, abs(r.e_d2[q] - e_d2[(x, y)]) / abs(e_d2[(x, y)]))
        worst = max(worst, _rel(r.e_m2, e_m2))
    ok &= worst < 1e-12
    return ok, f"worst relative difference {worst:.3e}"


@_safe
def pin_dense_solve(orc):
    """The converged iteration equals the LAPACK solution of the stacked linear
    system (all T_X and all ordered-pair Tau)."""
    worst = 0.0
    cases = [tiny(sizes=((2, 3), (2, 3))), tiny(sizes=((2, 3), (1, 4), (3, 2))),
             general_k(tiny(sizes=((2, 3), (3, 2), (2, 2))))]
    for p in cases:
        r = orc.solve(p, tol=1e-15, max_sweeps=200)
        T, tau, e_m2, e_d2 = _brute.dense_solve(p)
        if r.status != 0:
            return False, f"status {r.status}"
        for x in range(p.n_mono):
            worst = max(worst, _rel(r.T[x], T[x]))
        for q in range(p.n_pair):
            x, y = (int(t) for t in p.pairs[q])
            worst = max(worst, _rel(r.Tau[q], tau[(x, y)]))
            worst = max(worst, _rel(r.Tau[q].transpose(2, 3, 0, 1), tau[(y, x)]))
            worst = max(worst, abs(r.e_d2[q] - e_d2[(x, y)]) / abs(e_d2[(x, y)]))
        worst = max(worst, _rel(r.e_m2, e_m2))
    return worst < 1e-10, f"worst relative difference {worst:.3e}"


@_safe
def pin_relabel_and_orientation(orc):
    """Relabelling monomers and storing pairs reversed (V -> V^T) permutes the
    per-monomer results and leaves every energy unchanged."""
    p = tiny(sizes=((2, 3), (1, 4), (3, 2), (2, 2)))
    perm = np.array([2, 0, 3, 1])
    flip = np.arange(p.n_pair) % 2 == 0
    q = p.relabel(perm, flip)
    r0 = orc.solve(p, tol=1e-14)
    r1 = orc.solve(q, tol=1e-14)
    worst = abs(r0.e_total - r1.e_total) / abs(r0.e_total)
    worst = max(worst, _rel(r1.e_m2, r0.e_m2[perm]))
    worst = max(worst, _rel(r1.e_d2, r0.e_d2))
    for new, old in enumerate(perm):
        worst = max(worst, _rel(r1.T[new], r0.T[old]))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_sign_flip_bitwise(orc):
    """Negating V on any subset of pairs leaves T and all energies bitwise
    unchanged (Tau flips sign, v.Tau does not; IEEE negation is exact)."""
    p = tiny(sizes=((2, 3), (1, 4), (3, 2), (2, 2)))
    q = tiny(sizes=((2, 3), (1, 4), (3, 2), (2, 2)))
    for k in range(q.n_pair):
        if k % 3 != 1:
            q.v[q.v_off[k]:q.v_off[k + 1]] *= -1.0
    r0 = orc.solve(p, tol=0.0, max_sweeps=3)
    r1 = orc.solve(q, tol=0.0, max_sweeps=3)
    ok = all(np.array_equal(a, b) for a, b in zip(r0.T, r1.T))
    ok &= np.array_equal(r0.e_m2, r1.e_m2) and np.array_equal(r0.e_d2, r1.e_d2)
    return bool(ok), "bitwise" if ok else "differs"


@_safe
def pin_power_of_two_scaling_bitwise(orc):
    """(eps, K, V) -> 2^k (eps, K, V): T unchanged, every energy times 2^k, bitwise."""
    p = tiny()
    q = tiny()
    q.eps *= 8.0
    q.k *= 8.0
    q.v *= 8.0
    r0 = orc.solve(p, tol=0.0, max_sweeps=3)
    r1 = orc.solve(q, tol=0.0, max_sweeps=3)
    ok = all(np.array_equal(a, b) for a, b in zip(r0.T, r1.T))
    ok &= np.array_equal(8.0 * r0.e_m2, r1.e_m2) and np.array_equal(8.0 * r0.e_d2, r1.e_d2)
    return bool(ok), "bitwise" if ok else "differs"


@_safe
def pin_disconnected_additivity(orc):
    """Two clusters with no pairs between them: energies of the union are the
    energies of the separate solves."""
    a = tiny(cluster=1)
    b = tiny(sizes=((1, 3), (2, 2)), cluster=2)
    u = concat_problems([a, b])
    ra, rb, ru = (orc.solve(x, tol=1e-15) for x in (a, b, u))
    worst = _rel(ru.e_m2, np.concatenate([ra.e_m2, rb.e_m2]))
    worst = max(worst, _rel(ru.e_d2, np.concatenate([ra.e_d2, rb.e_d2])))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_orbital_permutation(orc):
    """Reordering the occupied and the virtual orbitals of one monomer
    consistently in eps, K and V leaves every energy unchanged."""
    p = tiny()
    q = tiny()
    x = 0
    o, v = int(p.n_occ[x]), int(p.n_vir[x])
    po = np.array([1, 0])
    pv = np.array([2, 0, 1])
    eo, ev = p.eps_of(x)
    q.eps[q.eps_off[x]:q.eps_off[x] + o] = eo[po]
    q.eps[q.eps_off[x] + o:q.eps_off[x + 1]] = ev[pv]
    q.k[q.k_off[x]:q.k_off[x + 1]] = p.k_of(x)[np.ix_(po, po, pv, pv)].ravel()
    for k in range(p.n_pair):
        X, Y = (int(t) for t in p.pairs[k])
        V = p.v_of(k)
        if X == x:
            V = V[np.ix_(po, pv, np.arange(V.shape[2]), np.arange(V.shape[3]))]
        elif Y == x:
            V = V[np.ix_(np.arange(V.shape[0]), np.arange(V.shape[1]), po, pv)]
        q.v[q.v_off[k]:q.v_off[k + 1]] = V.ravel()
    r0 = orc.solve(p, tol=1e-15)
    r1 = orc.solve(q, tol=1e-15)
    worst = max(_rel(r1.e_m2, r0.e_m2), _rel(r1.e_d2, r0.e_d2))
    return worst < 1e-12, f"worst relative difference {worst:.3e}"


@_safe
def pin_pair_symmetry(orc):
    """With K[i,j,a,b] = K[j,i,b,a] (real orbitals), the converged monomer
    amplitudes keep T[i,j,a,b] = T[j,i,b,a]."""
    p = tiny(sizes=((2, 3), (3, 2), (2, 2)))
    r = orc.solve(p, tol=1e-15)
    worst = max(_rel(t, t.transpose(1, 0, 3, 2)) for t in r.T)
    return worst < 1e-13, f"worst asymmetry {worst:.3e}"


@_safe
def pin_divergence_detected(orc):
    """At the literal coupling magnitude (scale 1) of the 2x2x2 crystal, the sweep
    map's dominant eigenvalue exceeds one: the iteration must report divergence."""
    p = make_workload("hf-2x2x2", coupling_scale=1.0)
    r = orc.solve(p, tol=1e-10, max_sweeps=60)
    return r.status == -5, f"status {r.status} after {r.sweeps} sweeps"


def coupling_only_dimer(sx, sy, seed, sigma=0.05):
    """Two monomers whose only nonzero two-electron integrals are the Coulomb
    integrals (ai|bj) between an occupied-virtual distribution of X and one of Y,
    cut from one real tensor (pq|rs) of the dimer's orbitals (every permutation
    of a real-orbital integral filled in).  The intramonomer block K is then zero
    and the reduced equations are the complete equations of this Hamiltonian.
    Returns (problem, g, orbital energies, orbital table)."""
    rng = np.random.default_rng(seed)
    (ox, vx), (oy, vy) = sx, sy
    nx, ny = ox + vx, oy + vy
    OX, VX = np.arange(ox), np.arange(ox, nx)
    OY, VY = nx + np.arange(oy), nx + np.arange(oy, ny)
    blk = rng.normal(0.0, sigma, size=(vx, ox, vy, oy))           # (a i|b j)
    g = np.zeros((nx + ny,) * 4)
    for (p_, q_), pq in (((VX, OX), blk), ((OX, VX), blk.transpose(1, 0, 2, 3))):
        for (r_, s_), rs in (((VY, OY), pq), ((OY, VY), pq.transpose(0, 1, 3, 2))):
            g[np.ix_(p_, q_, r_, s_)] = rs
            g[np.ix_(r_, s_, p_, q_)] = rs.transpose(2, 3, 0, 1)
    ex = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, ox)), np.sort(rng.uniform(0.2, 3.0, vx))])
    ey = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, oy)), np.sort(rng.uniform(0.2, 3.0, vy))])
    orbs = [(0, k < ox, k if k < ox else k - ox) for k in range(nx)] + \
           [(1, k < oy, k if k < oy else k - oy) for k in range(ny)]
    p = make_lattice_problem(cubic_sites(2, 1, 1), None, sizes=[sx, sy], workload=TEST_WORKLOAD)
    assert p.n_pair == 1 and tuple(p.pairs[0]) == (0, 1)
    p.eps[:] = np.concatenate([ex, ey])
    p.k[:] = 0.0
    p.v[:] = blk.transpose(1, 0, 3, 2).ravel()                      # V[i,a,j,b] = (ai|bj)
    return p, g, np.concatenate([ex, ey]), orbs


@_safe
def pin_restricted_lccd_coupling(orc):
    """On a dimer whose only integrals are the inter-monomer Coulomb class (K = 0),
    the reduced equations are complete, and the method is LCCD (Sec. II.A): the
    converged energy, T_X, T_Y (alpha-beta amplitudes) and Tau equal restricted
    spin-orbital LCCD solved densely in the excitations that keep each electron
    on its monomer.  Fixes the spin sum of the pair term of Eq. 58 (twice the
    printed term) and the 2T - T of Eq. 59 against textbook LCCD."""
    from .pins_dimer import compare_restricted_lccd
    worst = 0.0
    for sx, sy, seed in [((1, 2), (1, 2), 31), ((2, 2), (1, 3), 32), ((2, 3), (2, 2), 33)]:
        p, g, e, orbs = coupling_only_dimer(sx, sy, seed, sigma=0.15)
        r = orc.solve(p, tol=1e-15, max_sweeps=400)
        if r.status != 0:
            return False, f"status {r.status}"
        if not np.any(r.T[0]):
            return False, "no monomer amplitudes formed"
        worst = max(worst, compare_restricted_lccd(r, sx, sy, g, e, orbs))
    return worst < 1e-10, f"worst relative difference {worst:.3e}"


ALL_PINS = [
    pin_zero_coupling_mp2, pin_dispersion_mp2, pin_brute_force_sweeps,
    pin_dense_solve, pin_relabel_and_orientation, pin_sign_flip_bitwise,
    pin_power_of_two_scaling_bitwise, pin_disconnected_additivity, pin_orbital_permutation,
    pin_pair_symmetry, pin_restricted_lccd_coupling,
]
