"""Batched clusters (one resident batch, per-cluster stopping) and HIP-graph
captured sweeps, against solo solves and the FP64 oracle.

Each cluster of a batch follows the same sequence of operations as its solo
solve; the only difference is the order of the FP64 atomic additions into G,
so per-cluster energies agree with the solo ones to rounding (checked at
1e-12 relative) and sweep counts agree exactly.
"""
import numpy as np
import pytest

from oracle import mcpt_oracle
from synth import cluster_sites, make_cluster_batch, make_lattice_problem, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

SAME_RTOL = 1e-12      # batch or graph vs solo / eager (same arithmetic, atomics order aside)
ORACLE_RTOL = 1e-10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def clusters():
    """Uneven clusters: 3-20 monomers mixing o5v27 / o8v56, plus a lone monomer."""
    cl = make_cluster_batch(5, min_mono=3, max_mono=20, first=100)
    lone = make_lattice_problem(cluster_sites(1), 2.0, workload=4, cluster=99, mixed_sizes=True)
    return cl[:2] + [lone] + cl[2:]


def solo(ctx, prob, **opts):
    pid = ctx.upload(prob)
    s = ctx.run(pid, raise_on_error=False, **opts)
    e = ctx.energy(pid) if s["status"] != mc.MCPT_ERR_DIVERGED else None
    ctx.release(pid)
    return s, e


def check_against_solo(ctx, probs, **opts):
    print(f"[gpu] batch of {len(probs)} clusters sizes {[p.n_mono for p in probs]} {opts}", flush=True)
    pid = ctx.upload_batch(probs)
    s = ctx.run(pid, raise_on_error=False, **opts)
    per = ctx.cluster_results(pid)
    e = ctx.energy(pid)
    sl = ctx.cluster_slices(pid)
    ctx.release(pid)
    assert len(per) == len(probs)
    worst = mc.MCPT_OK
    for q, p in enumerate(probs):
        s1, e1 = solo(ctx, p, **opts)
        cq = per[q]
        assert cq["status"] == s1["status"], (q, cq, s1)
        assert cq["sweeps"] == s1["sweeps"], (q, cq["sweeps"], s1["sweeps"])
        assert cq["polish_sweeps"] == s1["polish_sweeps"]
        if cq["status"] == mc.MCPT_ERR_DIVERGED:
            worst = mc.MCPT_ERR_DIVERGED
            continue
        for k in ("e_total", "e_mono", "e_dimer", "e_mono0"):
            assert abs(cq[k] - s1[k]) <= SAME_RTOL * max(abs(s1[k]), 1e-300), (q, k, cq[k], s1[k])
        ms, ps = sl[q]
        assert rel(e["e_m2"][ms], e1["e_m2"]) <= SAME_RTOL
        assert rel(e["de_m2"][ms], e1["de_m2"]) <= 1e-9
        if p.n_pair:
            assert rel(e["e_d2"][ps], e1["e_d2"]) <= 1e-11
    assert s["status"] == worst
    if worst == mc.MCPT_OK:
        tot = sum(c["e_total"] for c in per)
        assert abs(s["e_total"] - tot) <= 1e-13 * abs(tot)
        assert s["sweeps"] == max(c["sweeps"] for c in per) or opts.get("precision", 0) != mc.MCPT_FP64
    return per


def test_batch_fp64_equals_solo_and_oracle(ctx, clusters):
    per = check_against_solo(ctx, clusters, tol=1e-10)
    for q in (0, 2):   # a small cluster and the lone monomer against the oracle
        r = mcpt_oracle.solve(clusters[q], tol=1e-10, max_sweeps=200)
        assert per[q]["sweeps"] == r.sweeps
        assert abs(per[q]["e_total"] - r.e_total) <= ORACLE_RTOL * abs(r.e_total)


@pytest.mark.parametrize("prec", [mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp32", "bf16"])
def test_batch_polish_equals_solo(ctx, clusters, prec):
    check_against_solo(ctx, clusters, tol=1e-10, precision=prec, polish=1)


def test_batch_reduced_precision_no_polish_equals_solo(ctx, clusters):
    check_against_solo(ctx, clusters, tol=1e-7, precision=mc.MCPT_FP32, polish=0)


def test_batch_fixed_sweeps_equals_solo(ctx, clusters):
    per = check_against_solo(ctx, clusters, tol=0.0, max_sweeps=4)
    assert all(c["sweeps"] == 4 for c in per)


def test_batch_diverging_cluster_does_not_stop_the_others(ctx, clusters):
    bad = make_workload("hf-2x2x2", coupling_scale=1.0)
    probs = [clusters[0], bad, clusters[3]]
    per = check_against_solo(ctx, probs, tol=1e-10, max_sweeps=60)
    assert per[1]["status"] == mc.MCPT_ERR_DIVERGED
    assert per[0]["status"] == mc.MCPT_OK and per[2]["status"] == mc.MCPT_OK


@pytest.mark.parametrize("prec,polish,every", [(mc.MCPT_FP64, 1, 1), (mc.MCPT_FP64, 1, 3),
                                               (mc.MCPT_FP32, 1, 1), (mc.MCPT_BF16, 1, 2),
                                               (mc.MCPT_FP32, 0, 3)],
                         ids=["fp64-k1", "fp64-k3", "fp32polish-k1", "bf16polish-k2", "fp32-k3"])
def test_graph_replay_equals_eager(ctx, clusters, prec, polish, every):
    """Captured sweeps replayed several times, with eager runs between the replays."""
    print(f"[gpu] graph prec={prec} polish={polish} every={every}", flush=True)
    tol = 1e-10 if polish or prec == mc.MCPT_FP64 else 1e-7
    opts = dict(tol=tol, precision=prec, polish=polish, check_every=every)
    pid = ctx.upload_batch(clusters)
    eager = ctx.run(pid, **opts)
    e0 = ctx.energy(pid)
    per0 = ctx.cluster_results(pid)
    for rep in range(3):
        g = ctx.run(pid, graph=1, **opts)
        eg = ctx.energy(pid)
        perg = ctx.cluster_results(pid)
        assert g["sweeps"] == eager["sweeps"] and g["polish_sweeps"] == eager["polish_sweeps"], (rep, g, eager)
        assert abs(g["e_total"] - eager["e_total"]) <= SAME_RTOL * abs(eager["e_total"])
        assert rel(eg["e_m2"], e0["e_m2"]) <= SAME_RTOL
        assert rel(eg["t"], e0["t"]) <= 1e-10
        assert [c["sweeps"] for c in perg] == [c["sweeps"] for c in per0]
        again = ctx.run(pid, **opts)   # eager work between replays
        assert again["sweeps"] == eager["sweeps"]
    ctx.release(pid)


def test_graph_fixed_sweeps_odd_count(ctx, clusters):
    """tol = 0 with an odd sweep cap: surplus captured sweeps must be no-ops."""
    pid = ctx.upload_batch(clusters)
    a = ctx.run(pid, tol=0.0, max_sweeps=5)
    ea = ctx.energy(pid)
    b = ctx.run(pid, tol=0.0, max_sweeps=5, graph=1, check_every=2)
    eb = ctx.energy(pid)
    ctx.release(pid)
    assert a["sweeps"] == b["sweeps"] == 5
    assert rel(eb["t"], ea["t"]) <= 1e-12
    assert abs(a["e_total"] - b["e_total"]) <= SAME_RTOL * abs(a["e_total"])


def test_options_rejected(ctx, clusters):
    pid = ctx.upload(clusters[0])
    for bad in (dict(deterministic=2), dict(graph=2)):
        with pytest.raises(mc.MCPTError) as ei:
            ctx.run(pid, tol=1e-10, **bad)
        assert ei.value.status == mc.MCPT_ERR_INVALID
    ctx.release(pid)
