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


def _by_sites(p):
    """Monomer inputs and pair blocks keyed by lattice sites (orientation-free)."""
    mono = {tuple(int(c) for c in p.sites[x]): (p.eps_of(x), p.k_of(x)) for x in range(p.n_mono)}
    pairs = {}
    for q, (x, y) in enumerate(p.pairs):
        sx, sy = tuple(int(c) for c in p.sites[x]), tuple(int(c) for c in p.sites[y])
        blk = p.v_of(q)
        if sx > sy:
            sx, sy, blk = sy, sx, blk.transpose(2, 3, 0, 1)
        pairs[(sx, sy)] = blk
    return mono, pairs


def test_served_stream_request_equals_a_displaced_lattice_of_its_sites():
    """A request of the prefix-relabelled stream is the crystal's own inputs on the
    n monomers nearest the centre, with the displaced monomer's blocks rescaled
    exactly as a from-scratch displaced lattice of those sites draws them."""
    from synth import ServedStream
    base = make_workload("hf-5x5x5-c2")
    w = WORKLOADS["hf-5x5x5-c2"]
    st = ServedStream(base)
    sites = np.asarray(base.sites)
    d2 = ((sites - sites.mean(axis=0)) ** 2).sum(axis=1)
    for r in (0, 5, 17):
        p = st.request(r)
        n, mono, axis, shift = st.draw(r)
        assert p.n_mono == n
        nearest = {tuple(int(c) for c in sites[x]) for x in np.lexsort((np.arange(len(sites)), d2))[:n]}
        assert {tuple(int(c) for c in s) for s in p.sites} == nearest
        # the generator keys a pair's draw by its sites in lexicographic order, as the crystal lists them
        lex = np.lexsort(np.asarray(p.sites)[:, ::-1].T)
        pos_of = np.empty(n, dtype=np.int64)
        pos_of[lex] = np.arange(n)
        ref = make_lattice_problem(np.asarray(p.sites)[lex], w["cutoff"], workload=w["workload"],
                                   displacement=(int(pos_of[mono]), axis, shift))
        (ma, pa), (mb, pb) = _by_sites(p), _by_sites(ref)
        assert ma.keys() == mb.keys() and pa.keys() == pb.keys()
        for key in ma:
            assert np.array_equal(ma[key][0][0], mb[key][0][0]) and np.array_equal(ma[key][1], mb[key][1])
        for key in pa:
            assert np.allclose(pa[key], pb[key], rtol=1e-14, atol=0.0), key


def test_served_stream_lend_equals_request_and_restores():
    from synth import ServedStream
    base = make_workload("hf-5x5x5-c2")
    st = ServedStream(base)
    before = st.v.copy()
    for r in (2, 9):
        ref = st.request(r)
        with st.lend(r) as p:
            for f in ("n_occ", "n_vir", "eps", "k", "pairs", "v"):
                assert np.array_equal(getattr(p, f), getattr(ref, f)), f
        assert np.array_equal(st.v, before)
