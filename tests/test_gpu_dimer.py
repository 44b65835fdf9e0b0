"""Dimer-internal terms of Eq. 59 (ladders, cross rings, monomer rings, Tau
iterated) on the GPU against the oracle: fixed sweep counts element by element
on uniform clusters of one to nine MFMA tiles per edge (n = 6, 51, 135, the
last two with ragged tails), with physical-symmetry and with general
integrals, monomers at and above the LDS limit of the staged pair ladder (up to
o8v56, n = 448), pairs of monomers of different sizes, the converged solve with
equal sweep counts, graph replay, and the error paths.  Bar: 1e-10 relative (FP64), sweep counts equal."""
import json
import os
import types

import numpy as np
import pytest

from oracle import mcpt_dimer
from synth import (LCCD_K_SCALE, concat_lccd, cubic_sites, dimer_integrals, lccd_integrals, make_dimer_workload,
                   make_lattice_problem)
import paper_1409_2700_amd as mc
from paper_1409_2700_amd import mcpt as binding

pytestmark = pytest.mark.gpu

TOL = 1e-10
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def flat_t(r):
    return np.concatenate([t.ravel() for t in r.T])


def cluster(o, v, dims=(2, 2, 1), scale=0.5, workload=940, general=False):
    p = make_lattice_problem(cubic_sites(*dims), None, o=o, v=v, workload=workload, coupling_scale=scale,
                             k_scale=LCCD_K_SCALE)
    ints = lccd_integrals(p)
    dints = dimer_integrals(p)
    if general:   # no permutational symmetry in any dimer class
        rng = np.random.default_rng(workload)
        for arr in (dints.w, dints.q, dints.cx, dints.cy):
            arr[:] = rng.normal(0.0, 0.01, size=arr.shape)
    return p, ints, dints


def run_gpu(ctx, p, ints, dints, **opts):
    pid = ctx.upload(p)
    ctx.lccd_attach(pid, ints)
    ctx.dimer_attach(pid, dints)
    s = ctx.run(pid, raise_on_error=False, **opts)
    s["error"] = binding.last_error() if s["return"] != mc.MCPT_OK else ""
    e = None
    if s["return"] in (mc.MCPT_OK, mc.MCPT_ERR_NOT_CONVERGED):
        e = ctx.energy(pid)
        e["tau"] = ctx.dimer_tau(pid)
    ctx.release(pid)
    return s, e


def flat_tau(r):
    return np.concatenate([np.asarray(t).ravel() for t in r.Tau])


@pytest.mark.parametrize("o,v,general,sweeps", [(2, 3, False, 1), (2, 3, True, 3), (3, 17, False, 2),
                                                (3, 17, True, 2), (5, 27, False, 2), (5, 27, True, 3)])
def test_fixed_sweeps_elementwise(ctx, o, v, general, sweeps):
    p, ints, dints = cluster(o, v, general=general)
    print(f"[gpu] dimer fixed sweeps={sweeps} o={o} v={v} general={general} P={p.n_pair}", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=0.0, max_sweeps=sweeps)
    s, e = run_gpu(ctx, p, ints, dints, tol=0.0, max_sweeps=sweeps)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert s["sweeps"] == sweeps
    assert rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL      # every dimer amplitude, element by element
    assert rel(e["e_m2"], ref.e_m2) <= TOL
    assert rel(e["e_d2"], ref.e_d2) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)


@pytest.mark.parametrize("graph", [0, 1])
def test_converged_matches_oracle(ctx, graph):
    p, ints, dints = cluster(5, 27, dims=(3, 1, 1), workload=941)
    print(f"[gpu] dimer converged graph={graph} P={p.n_pair}", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=TOL, max_sweeps=200)
    s, e = run_gpu(ctx, p, ints, dints, tol=TOL, max_sweeps=200, graph=graph)
    assert ref.status == 0 and s["return"] == mc.MCPT_OK, s["error"]
    assert s["sweeps"] == ref.sweeps
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL and rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)


def test_errors_and_detach(ctx):
    p, ints, dints = cluster(2, 3)
    pid = ctx.upload(p)
    with pytest.raises(mc.MCPTError):              # needs the intramonomer integrals
        ctx.dimer_attach(pid, dints)
    ctx.lccd_attach(pid, ints)
    ctx.dimer_attach(pid, dints)
    s = ctx.run(pid, raise_on_error=False, precision=mc.MCPT_FP32)
    assert s["return"] == mc.MCPT_ERR_INVALID       # FP64 only
    ctx.dimer_attach(pid, None)                     # detached: the full monomer equation alone
    s = ctx.run(pid, tol=0.0, max_sweeps=2)
    from oracle import mcpt_lccd
    ref = mcpt_lccd.solve(p, ints, tol=0.0, max_sweeps=2)
    assert rel(ctx.energy(pid)["e_d2"], ref.e_d2) <= TOL
    ctx.release(pid)


def mixed_cluster(sizes, dims, scale=0.5, workload=961, general=False):
    p = make_lattice_problem(cubic_sites(*dims), None, sizes=list(sizes), workload=workload, coupling_scale=scale,
                             k_scale=LCCD_K_SCALE)
    ints = lccd_integrals(p)
    dints = dimer_integrals(p)
    if general:
        rng = np.random.default_rng(workload)
        for arr in (dints.w, dints.q, dints.cx, dints.cy):
            arr[:] = rng.normal(0.0, 0.01, size=arr.shape)
    return p, ints, dints


@pytest.mark.parametrize("general,sweeps", [(False, 1), (False, 3), (True, 2)])
def test_mixed_sizes_fixed_sweeps(ctx, general, sweeps):
    """Pairs of monomers of different sizes (X smaller or larger than Y, one side
    o8v56 beyond the LDS-staged ladder): every T, every pair's Tau and the energies
    element by element against the oracle."""
    sizes = ((2, 3), (5, 27), (8, 56), (3, 17))
    p, ints, dints = mixed_cluster(sizes, (2, 2, 1), general=general)
    print(f"[gpu] dimer mixed sizes {sizes} P={p.n_pair} sweeps={sweeps} general={general}", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=0.0, max_sweeps=sweeps)
    s, e = run_gpu(ctx, p, ints, dints, tol=0.0, max_sweeps=sweeps)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)


def test_mixed_sizes_converged(ctx):
    sizes = ((5, 27), (3, 17), (5, 27), (2, 9), (4, 11))
    p, ints, dints = mixed_cluster(sizes, (5, 1, 1), scale=0.3, workload=962)
    print(f"[gpu] dimer mixed sizes converged P={p.n_pair}", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=TOL, max_sweeps=200)
    s, e = run_gpu(ctx, p, ints, dints, tol=TOL, max_sweeps=200)
    assert ref.status == 0 and s["return"] == mc.MCPT_OK, s["error"]
    assert s["sweeps"] == ref.sweeps
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)


def test_batch_equals_solo(ctx):
    """Two clusters of one batch stop on their own residuals exactly as alone."""
    a = cluster(2, 3, workload=950)
    b = cluster(2, 3, dims=(3, 1, 1), workload=951)
    solo = [run_gpu(ctx, *c, tol=TOL, max_sweeps=200)[0] for c in (a, b)]
    pid = ctx.upload_batch([a[0], b[0]])
    ctx.lccd_attach(pid, concat_lccd([a[1], b[1]]))
    ctx.dimer_attach(pid, types.SimpleNamespace(**{k: np.concatenate([getattr(a[2], k), getattr(b[2], k)])
                                                   for k in ("w", "q", "cx", "cy")}))
    s = ctx.run(pid, tol=TOL, max_sweeps=200)
    res = ctx.cluster_results(pid)
    ctx.release(pid)
    assert s["return"] == mc.MCPT_OK
    for k in range(2):
        assert res[k]["sweeps"] == solo[k]["sweeps"]
        assert abs(res[k]["e_total"] - solo[k]["e_total"]) <= 1e-12 * abs(solo[k]["e_total"])


@pytest.mark.parametrize("name", ["hf-3x3x3-c1", "hf-10x10x10-c1", "hf-10x10x10-c1.5"])
def test_converged_crystals_match_stored_oracle(ctx, name):
    with open(os.path.join(GOLDEN, f"dimer-{name}.json")) as f:
        g = json.load(f)
    p, ints, dints = make_dimer_workload(name, workers=min(16, os.cpu_count() or 1))
    print(f"[gpu] dimer converged {name} N={p.n_mono} P={p.n_pair}", flush=True)
    s, e = run_gpu(ctx, p, ints, dints, tol=g["tol"], max_sweeps=400, check_every=4)
    assert s["return"] == mc.MCPT_OK and g["status"] == 0, s["error"]
    assert s["sweeps"] == g["sweeps"]
    assert abs(s["e_total"] - g["e_total"]) <= TOL * abs(g["e_total"])
    assert abs(s["e_mono0"] - g["e_lccd_total"]) <= TOL * abs(g["e_lccd_total"])
    assert rel(e["e_m2"], g["e_m2"]) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], g["e_lccd"]) <= TOL
    assert rel(e["e_d2"][g["pair_index"]], g["e_d2"]) <= TOL


def test_device_integrals(ctx):
    """Dimer classes handed over in device memory give the host hand-over's results."""
    import ctypes
    hip = ctypes.CDLL(os.path.join("/opt/rocm/lib", "libamdhip64.so"))
    p, ints, dints = cluster(3, 17, workload=952)
    pid = ctx.upload(p)
    ctx.lccd_attach(pid, ints)
    ctx.dimer_attach(pid, dints)
    a = ctx.run(pid, tol=TOL)
    ea = ctx.energy(pid)
    arrs = [np.ascontiguousarray(x) for x in (dints.w, dints.q, dints.cx, dints.cy)]
    ptrs = []
    try:
        for arr in arrs:
            d = ctypes.c_void_p()
            assert hip.hipMalloc(ctypes.byref(d), ctypes.c_size_t(max(arr.nbytes, 8))) == 0
            ptrs.append(d)
            assert hip.hipMemcpy(d, arr.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(arr.nbytes), 1) == 0
        ctx.dimer_attach(pid, None, device_ptrs=tuple(d.value for d in ptrs))
        b = ctx.run(pid, tol=TOL)
        eb = ctx.energy(pid)
    finally:
        for d in ptrs:
            hip.hipFree(d)
    ctx.release(pid)
    assert a["return"] == mc.MCPT_OK and a["sweeps"] == b["sweeps"]
    assert rel(eb["e_m2"], ea["e_m2"]) <= 1e-13 and rel(eb["e_d2"], ea["e_d2"]) <= 1e-13


def test_single_pair_and_no_pairs(ctx):
    """One pair (two monomers) against the oracle; a problem without pairs is refused."""
    p, ints, dints = cluster(5, 27, dims=(2, 1, 1), workload=953)
    ref = mcpt_dimer.solve(p, ints, dints, tol=0.0, max_sweeps=3)
    s, e = run_gpu(ctx, p, ints, dints, tol=0.0, max_sweeps=3)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["t"], flat_t(ref)) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    q = make_lattice_problem(cubic_sites(1, 1, 1), None, o=2, v=3, workload=954)
    pid = ctx.upload(q)
    ctx.lccd_attach(pid, lccd_integrals(q))
    with pytest.raises(mc.MCPTError):
        ctx.dimer_attach(pid, dimer_integrals(q))
    ctx.release(pid)


@pytest.mark.parametrize("o,v,workload", [(6, 23, 955), (6, 24, 956), (8, 56, 958)])
def test_monomers_at_and_above_the_lds_limit(ctx, o, v, workload):
    """o = 6, v = 23 (n = 138): the largest pair whose Tau fits the LDS-staged ladder
    (three column tiles per task, 155 KB of the 160 KiB); o = 6, v = 24 (n = 144) and
    o = 8, v = 56 (n = 448, four column tiles, 79 MB of W_XY per pair) run the pair
    ladder from global memory.  Element by element after two sweeps."""
    p, ints, dints = cluster(o, v, dims=(2, 1, 1), workload=workload)
    print(f"[gpu] dimer o={o} v={v} n={o * v} fixed sweeps", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=0.0, max_sweeps=2)
    s, e = run_gpu(ctx, p, ints, dints, tol=0.0, max_sweeps=2)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["t"], flat_t(ref)) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL
    assert rel(e["e_m2"], ref.e_m2) <= TOL


def test_o8v56_converged_and_too_large_refused(ctx):
    """The o8v56 pair (at the crystal's coupling scale, where its monomer equations
    converge) with the oracle's sweep count; o = 9 is refused (by the intramonomer
    terms, which the dimer terms need)."""
    p, ints, dints = cluster(8, 56, dims=(2, 1, 1), scale=0.18, workload=959)
    print("[gpu] dimer o8v56 converged", flush=True)
    ref = mcpt_dimer.solve(p, ints, dints, tol=TOL, max_sweeps=200)
    s, e = run_gpu(ctx, p, ints, dints, tol=TOL, max_sweeps=200)
    assert ref.status == 0 and s["return"] == mc.MCPT_OK, s["error"]
    assert s["sweeps"] == ref.sweeps
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["tau"], flat_tau(ref)) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)
    q, qi, qd = cluster(9, 3, dims=(2, 1, 1), workload=960)
    pid = ctx.upload(q)
    with pytest.raises(mc.MCPTError):
        ctx.lccd_attach(pid, qi)
    with pytest.raises(mc.MCPTError):
        ctx.dimer_attach(pid, qd)
    ctx.release(pid)


def test_lccd_reattach_detaches_dimer_terms(ctx):
    """Attaching the intramonomer integrals again drops the dimer classes: the run
    is the full monomer equation's, and the dimer terms can be attached again."""
    from oracle import mcpt_lccd
    p, ints, dints = cluster(3, 17, workload=957)
    pid = ctx.upload(p)
    ctx.lccd_attach(pid, ints)
    ctx.dimer_attach(pid, dints)
    ctx.lccd_attach(pid, ints)
    s = ctx.run(pid, tol=0.0, max_sweeps=2)
    e = ctx.energy(pid)
    ref = mcpt_lccd.solve(p, ints, tol=0.0, max_sweeps=2)
    assert s["return"] == mc.MCPT_OK and rel(e["e_d2"], ref.e_d2) <= TOL
    ctx.dimer_attach(pid, dints)
    s = ctx.run(pid, tol=0.0, max_sweeps=2)
    e = ctx.energy(pid)
    ctx.release(pid)
    ref = mcpt_dimer.solve(p, ints, dints, tol=0.0, max_sweeps=2)
    assert s["return"] == mc.MCPT_OK and rel(e["e_d2"], ref.e_d2) <= TOL and rel(e["t"], flat_t(ref)) <= TOL
