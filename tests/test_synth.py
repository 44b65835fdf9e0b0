"""The seeded input generators: the carved served requests are exactly the
crystal's own inputs restricted to the carved monomers, with the displaced
monomer's pair blocks rescaled as a from-scratch displaced lattice has them."""
import numpy as np

from synth import carve_served_request, make_lattice_problem, make_workload, WORKLOADS


def test_carving_the_whole_crystal_equals_a_displaced_lattice():
    base = make_workload("hf-2x2x2")
    p = carve_served_request(base, 3, min_mono=8, max_mono=8)
    w = WORKLOADS["hf-2x2x2"]
    ref = make_lattice_problem(base.sites, w["cutoff"], workload=w["workload"], displacement=p.meta["displacement"])
    for f in ("n_occ", "n_vir", "eps", "k", "pairs", "v"):
        assert np.array_equal(getattr(p, f), getattr(ref, f)), f
    assert not np.array_equal(p.v, base.v)


def test_carved_subcluster_keeps_blocks_of_its_pairs():
    base = make_workload("hf-5x5x5-c2")
    p = carve_served_request(base, 11, min_mono=20, max_mono=20)
    assert p.n_mono == 20
    # map back: every carved monomer is a base monomer with the same site and inputs
    idx = [int(np.flatnonzero((base.sites == s).all(axis=1))[0]) for s in p.sites]
    for a, x in enumerate(idx):
        assert np.array_equal(p.eps_of(a)[0], base.eps_of(x)[0]) and np.array_equal(p.k_of(a), base.k_of(x))
    d = p.meta["displacement"][0]
    base_pair = {(int(x), int(y)): q for q, (x, y) in enumerate(base.pairs)}
    for q, (x, y) in enumerate(p.pairs):
        bq = base_pair[(idx[x], idx[y])]
        if d not in (x, y):
            assert np.array_equal(p.v_of(q), base.v_of(bq))
        else:
            ratio = p.v_of(q) / base.v_of(bq)
            assert np.allclose(ratio, ratio.flat[0]) and abs(ratio.flat[0] - 1.0) < 0.01
    # every base pair between carved monomers is kept
    carved = set(idx)
    n_inside = sum(1 for (x, y) in base.pairs if x in carved and y in carved)
    assert n_inside == p.n_pair


def test_dimer_integrals_seeded_and_symmetric():
    """The dimer classes are keyed by the two sites (a pair drawn inside a larger
    crystal equals the same pair drawn alone) and symmetric within each charge
    distribution, (pq|rs) = (qp|rs) = (pq|sr)."""
    import numpy as np
    from synth import cubic_sites, dimer_integrals, make_lattice_problem
    big = make_lattice_problem(cubic_sites(3, 1, 1), 1.0, o=2, v=3, workload=930)
    small = make_lattice_problem(cubic_sites(2, 1, 1), 1.0, o=2, v=3, workload=930)
    db, ds = dimer_integrals(big), dimer_integrals(small)
    assert tuple(big.pairs[0]) == tuple(small.pairs[0]) == (0, 1)
    for f in ("w_of", "q_of", "cx_of", "cy_of"):
        assert np.array_equal(getattr(db, f)(0), getattr(ds, f)(0))
    w = db.w_of(1)                                   # [a, b, a1, b1] = (a a1|b b1)
    assert np.allclose(w, w.transpose(2, 1, 0, 3)) and np.allclose(w, w.transpose(0, 3, 2, 1))
    q = db.q_of(1)                                   # [i1, j1, i, j] = (i1 i|j1 j)
    assert np.allclose(q, q.transpose(2, 1, 0, 3)) and np.allclose(q, q.transpose(0, 3, 2, 1))
    for c in (db.cx_of(1), db.cy_of(1)):             # (i1 i|b b1), (j1 j|a a1)
        assert np.allclose(c, c.transpose(1, 0, 2, 3)) and np.allclose(c, c.transpose(0, 1, 3, 2))
    assert not np.allclose(db.w_of(0), db.w_of(1))
