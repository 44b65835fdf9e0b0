"""Full monomer equation (Eq. 58 with its intramonomer terms, isolated LCCD of
step 5) on the GPU against the oracle: fixed sweep counts element by element
on ragged clusters (one to several MFMA tiles per edge, o up to 8, v up to 56)
with physical-symmetry and with general integrals, the converged cubes (the
1000-monomer cube at full size against the stored oracle results), batches and
graph replay against plain runs, device-resident integrals, detaching, and the
error paths.  Bar: 1e-10 relative (FP64), sweep counts equal."""
import ctypes
import json
import os

import numpy as np
import pytest

from oracle import mcpt_lccd
from synth import (LCCD_K_SCALE, concat_lccd, cubic_sites, lccd_integrals, make_cluster_batch,
                   make_lattice_problem, make_lccd_workload)
import paper_1409_2700_amd as mc
from paper_1409_2700_amd import mcpt as binding

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = 1e-10


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def flat_t(r):
    return np.concatenate([t.ravel() for t in r.T]) if r.T else np.zeros(0)


def ragged(sizes=((2, 3), (5, 27), (3, 17), (1, 1), (8, 56), (4, 9)), scale=0.5, workload=920, general=False):
    p = make_lattice_problem(cubic_sites(len(sizes), 1, 1), None, sizes=list(sizes), workload=workload,
                             coupling_scale=scale, k_scale=LCCD_K_SCALE)
    ints = lccd_integrals(p)
    if general:
        rng = np.random.default_rng(workload)
        for x in range(p.n_mono):
            g = rng.normal(0.0, 0.01, size=p.k_of(x).shape)
            p.k[p.k_off[x]:p.k_off[x + 1]] = (g + g.transpose(1, 0, 3, 2)).ravel()
        ints.w[:] = rng.normal(0.0, 0.01, size=ints.w.shape)
        ints.q[:] = rng.normal(0.0, 0.01, size=ints.q.shape)
        ints.j[:] = rng.normal(0.0, 0.01, size=ints.j.shape)
    return p, ints


def run_gpu(ctx, p, ints, **opts):
    pid = ctx.upload(p)
    ctx.lccd_attach(pid, ints)
    s = ctx.run(pid, raise_on_error=False, **opts)
    s["error"] = binding.last_error() if s["return"] != mc.MCPT_OK else ""
    e = ctx.energy(pid) if s["return"] in (mc.MCPT_OK, mc.MCPT_ERR_NOT_CONVERGED) else None
    ctx.release(pid)
    return s, e


@pytest.mark.parametrize("general,sweeps", [(False, 0), (False, 1), (False, 3), (True, 2)])
def test_fixed_sweeps_elementwise(ctx, general, sweeps):
    p, ints = ragged(general=general)
    print(f"[gpu] lccd fixed sweeps={sweeps} general={general} N={p.n_mono} P={p.n_pair}", flush=True)
    ref = mcpt_lccd.solve(p, ints, tol=0.0, max_sweeps=sweeps)
    s, e = run_gpu(ctx, p, ints, tol=0.0, max_sweeps=sweeps)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert s["sweeps"] == sweeps and s["iso_sweeps"] == sweeps
    assert rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["e_m2"], ref.e_m2) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL       # E_LCCD of step 5
    assert rel(e["e_d2"], ref.e_d2) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)
    assert abs(s["e_mono0"] - ref.e_mono0) <= TOL * abs(ref.e_mono0)


@pytest.mark.parametrize("general", [False, True])
def test_fixed_sweeps_lds_staged_ladder(ctx, general):
    """Monomers whose amplitudes fit one workgroup's LDS (o v <= 135 here): the
    ladder kernel that stages T in LDS; element by element after 2 sweeps."""
    p, ints = ragged(sizes=((2, 3), (5, 27), (3, 17), (1, 1), (4, 9), (5, 27)), general=general, workload=921)
    ref = mcpt_lccd.solve(p, ints, tol=0.0, max_sweeps=2)
    s, e = run_gpu(ctx, p, ints, tol=0.0, max_sweeps=2)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["e_m2"], ref.e_m2) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL


def test_converged_ragged(ctx):
    p, ints = ragged(scale=0.5)
    ref = mcpt_lccd.solve(p, ints, tol=TOL, max_sweeps=300)
    s, e = run_gpu(ctx, p, ints, tol=TOL, max_sweeps=300)
    assert ref.status == 0 and s["return"] == mc.MCPT_OK
    assert s["sweeps"] == ref.sweeps
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL


@pytest.mark.parametrize("name", ["hf-2x2x2", "hf-5x5x5-c2", "hf-10x10x10-c3"])
def test_converged_cubes_match_stored_oracle(ctx, name):
    path = os.path.join(GOLDEN, f"lccd-{name}.json")
    with open(path) as f:
        g = json.load(f)
    p, ints = make_lccd_workload(name)
    print(f"[gpu] lccd converged {name} N={p.n_mono} P={p.n_pair}", flush=True)
    s, e = run_gpu(ctx, p, ints, tol=g["tol"], max_sweeps=400, check_every=4)
    assert s["return"] == mc.MCPT_OK and g["status"] == 0
    assert s["iso_sweeps"] == g["iso_sweeps"] and s["sweeps"] == g["sweeps"]
    assert abs(s["e_total"] - g["e_total"]) <= TOL * abs(g["e_total"])
    assert abs(s["e_mono0"] - g["e_lccd_total"]) <= TOL * abs(g["e_lccd_total"])
    assert rel(e["e_m2"], g["e_m2"]) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], g["e_lccd"]) <= TOL
    assert rel(e["e_d2"][g["pair_index"]], g["e_d2"]) <= TOL


@pytest.mark.parametrize("precision", [mc.MCPT_FP32, mc.MCPT_BF16])
@pytest.mark.parametrize("graph", [0, 1])
def test_mixed_precision_polish_matches_oracle(ctx, precision, graph):
    """Reduced-precision pair products with FP64 defect correction (the
    intramonomer terms of each correction applied in FP64): converged to the FP64
    tolerance, so within the FP64 bar of the oracle."""
    p, ints = ragged(sizes=((2, 3), (5, 27), (3, 17), (1, 1), (4, 9), (5, 27)), workload=922)
    ref = mcpt_lccd.solve(p, ints, tol=TOL, max_sweeps=300)
    s, e = run_gpu(ctx, p, ints, tol=TOL, max_sweeps=300, precision=precision, polish=1, graph=graph,
                   check_every=2)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL
    assert abs(s["e_total"] - ref.e_total) <= TOL * abs(ref.e_total)
    assert s["polish_sweeps"] < ref.sweeps


def test_mixed_precision_polish_cube(ctx):
    with open(os.path.join(GOLDEN, "lccd-hf-5x5x5-c2.json")) as f:
        g = json.load(f)
    p, ints = make_lccd_workload("hf-5x5x5-c2")
    s, e = run_gpu(ctx, p, ints, tol=g["tol"], max_sweeps=400, precision=mc.MCPT_BF16, polish=1)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert s["iso_sweeps"] == g["iso_sweeps"]
    assert abs(s["e_total"] - g["e_total"]) <= TOL * abs(g["e_total"])
    assert rel(e["e_m2"], g["e_m2"]) <= TOL and rel(e["e_m2"] - e["de_m2"], g["e_lccd"]) <= TOL


def test_no_pairs_shift_is_zero(ctx):
    p, ints = ragged()
    q = p.subset_pairs(np.zeros(p.n_pair, dtype=bool))
    ref = mcpt_lccd.solve(q, ints, tol=1e-12, max_sweeps=300)
    s, e = run_gpu(ctx, q, ints, tol=1e-12, max_sweeps=300)
    assert s["sweeps"] == s["iso_sweeps"] == ref.sweeps
    assert rel(e["e_m2"], ref.e_m2) <= TOL
    assert np.max(np.abs(e["de_m2"])) <= 1e-13 * np.max(np.abs(e["e_m2"]))


def test_batch_and_graph_equal_plain(ctx):
    probs = make_cluster_batch(3, min_mono=3, max_mono=12, first=720, mixed_sizes=True)
    for p in probs:
        p.k *= LCCD_K_SCALE
    ints = [lccd_integrals(p) for p in probs]
    solo = [run_gpu(ctx, p, i, tol=TOL, max_sweeps=300) for p, i in zip(probs, ints)]
    pid = ctx.upload_batch(probs)
    ctx.lccd_attach(pid, concat_lccd(ints))
    s = ctx.run(pid, tol=TOL, max_sweeps=300)
    e = ctx.energy(pid)
    per = ctx.cluster_results(pid)
    sl = ctx.cluster_slices(pid)
    g = ctx.run(pid, tol=TOL, max_sweeps=300, graph=1, check_every=3)
    eg = ctx.energy(pid)
    ctx.release(pid)
    for q, ((ss, es), pq) in enumerate(zip(solo, per)):
        assert pq["sweeps"] == ss["sweeps"] and pq["iso_sweeps"] == ss["iso_sweeps"], q
        assert rel(e["e_m2"][sl[q][0]], es["e_m2"]) <= 1e-12, q
        assert rel(e["de_m2"][sl[q][0]], es["de_m2"]) <= 1e-12, q
    assert g["sweeps"] == s["sweeps"] and g["iso_sweeps"] == s["iso_sweeps"]
    assert rel(eg["e_m2"], e["e_m2"]) <= 1e-12 and rel(eg["t"], e["t"]) <= 1e-12


def test_device_integrals_and_detach(ctx):
    hip = ctypes.CDLL(os.path.join("/opt/rocm/lib", "libamdhip64.so"))
    p, ints = ragged(sizes=((2, 3), (5, 27), (3, 17)))
    pid = ctx.upload(p)
    plain = ctx.run(pid, tol=TOL)
    ctx.lccd_attach(pid, ints)
    a = ctx.run(pid, tol=TOL)
    ea = ctx.energy(pid)
    arrs = [np.ascontiguousarray(x) for x in (ints.w, ints.q, ints.j)]
    ptrs = []
    try:
        for arr in arrs:
            d = ctypes.c_void_p()
            assert hip.hipMalloc(ctypes.byref(d), ctypes.c_size_t(max(arr.nbytes, 8))) == 0
            ptrs.append(d)
            assert hip.hipMemcpy(d, arr.ctypes.data_as(ctypes.c_void_p), ctypes.c_size_t(arr.nbytes), 1) == 0
        ctx.lccd_attach(pid, None, device_ptrs=tuple(d.value for d in ptrs))
        b = ctx.run(pid, tol=TOL)
        eb = ctx.energy(pid)
    finally:
        for d in ptrs:
            hip.hipFree(d)
    ctx.lccd_attach(pid, None)
    c = ctx.run(pid, tol=TOL)
    ctx.release(pid)
    assert a["sweeps"] == b["sweeps"] and rel(eb["e_m2"], ea["e_m2"]) <= 1e-13
    assert c["sweeps"] == plain["sweeps"] and c["iso_sweeps"] == 0
    assert abs(c["e_total"] - plain["e_total"]) <= 1e-13 * abs(plain["e_total"])


def test_errors(ctx):
    p, ints = ragged(sizes=((2, 3), (3, 4)))
    pid = ctx.upload(p)
    bad = lccd_integrals(p)
    bad.w[3] = np.inf
    with pytest.raises(mc.MCPTError) as ei:
        ctx.lccd_attach(pid, bad)
    assert ei.value.status == mc.MCPT_ERR_NONFINITE
    ctx.lccd_attach(pid, ints)
    r = ctx.run(pid, tol=TOL, raise_on_error=False, deterministic=1)
    assert r["return"] == mc.MCPT_ERR_INVALID
    r = ctx.run(pid, tol=TOL, max_sweeps=3, raise_on_error=False)
    assert r["return"] == mc.MCPT_ERR_NOT_CONVERGED and r["sweeps"] == 3
    with pytest.raises(mc.MCPTError) as ei:
        ctx.lccd_attach(pid + 10**6, ints)
    assert ei.value.status == mc.MCPT_ERR_UNKNOWN_ID
    ctx.release(pid)
    for sizes in (((1, 65),), ((9, 3),)):   # v above 64, o above 8
        wide, wi = ragged(sizes=sizes)
        pid = ctx.upload(wide)
        with pytest.raises(mc.MCPTError) as ei:
            ctx.lccd_attach(pid, wi)
        assert ei.value.status == mc.MCPT_ERR_INVALID
        ctx.release(pid)


def test_step5_divergence_detected(ctx):
    p, ints = ragged(sizes=((2, 3), (3, 4)))
    ints.w *= 400.0
    ref_e, _, st, res = mcpt_lccd.isolated_lccd(p, ints, tol=TOL, max_sweeps=200)
    s, _ = run_gpu(ctx, p, ints, tol=TOL, max_sweeps=200)
    assert st == mc.MCPT_ERR_DIVERGED
    assert s["return"] == mc.MCPT_ERR_DIVERGED


def test_relabelling_and_power_of_two_scaling(ctx):
    """Monomers relabelled with every other pair stored reversed give the same
    energies (permuted); eps and every integral times 8 give T unchanged and
    energies times 8 (to rounding: the pair contributions are added by atomics)."""
    p, ints = ragged(sizes=((2, 3), (5, 27), (3, 17), (4, 9)), workload=923)
    perm = np.array([2, 0, 3, 1])
    q = p.relabel(perm, np.arange(p.n_pair) % 2 == 0)
    s0, e0 = run_gpu(ctx, p, ints, tol=1e-12, max_sweeps=300)
    s1, e1 = run_gpu(ctx, q, ints.subset(perm), tol=1e-12, max_sweeps=300)
    assert s0["return"] == s1["return"] == mc.MCPT_OK
    assert abs(s1["e_total"] - s0["e_total"]) <= 1e-12 * abs(s0["e_total"])
    assert rel(e1["e_m2"], e0["e_m2"][perm]) <= 1e-12 and rel(e1["de_m2"], e0["de_m2"][perm]) <= 1e-10
    p8, i8 = ragged(sizes=((2, 3), (5, 27), (3, 17), (4, 9)), workload=923)
    for a in (p8.eps, p8.k, p8.v, i8.w, i8.q, i8.j):
        a *= 8.0
    s8, e8 = run_gpu(ctx, p8, i8, tol=0.0, max_sweeps=4)
    s0f, e0f = run_gpu(ctx, p, ints, tol=0.0, max_sweeps=4)
    assert rel(e8["t"], e0f["t"]) <= 1e-13
    assert rel(e8["e_m2"], 8.0 * e0f["e_m2"]) <= 1e-13 and rel(e8["e_d2"], 8.0 * e0f["e_d2"]) <= 1e-13


def test_largest_supported_monomer(ctx):
    """The size limits of the full monomer equation: o = 8 (64 hole pairs, four
    column tiles) and v = 64 (v^2 = 4096 columns, the whole offset table; o v =
    512, 32 tiles per edge with a ragged super-block row), beside the smallest
    monomer; one sweep element by element."""
    p, ints = ragged(sizes=((8, 64), (1, 1), (5, 27)), scale=0.3, workload=924)
    print(f"[gpu] lccd largest monomer N={p.n_mono} P={p.n_pair}", flush=True)
    ref = mcpt_lccd.solve(p, ints, tol=0.0, max_sweeps=1)
    s, e = run_gpu(ctx, p, ints, tol=0.0, max_sweeps=1)
    assert s["return"] == mc.MCPT_OK, s["error"]
    assert rel(e["t"], flat_t(ref)) <= TOL
    assert rel(e["e_m2"], ref.e_m2) <= TOL and rel(e["e_d2"], ref.e_d2) <= TOL
    assert rel(e["e_m2"] - e["de_m2"], ref.e_m2_0) <= TOL
