"""Deterministic mode: with `deterministic = 1` every pair stores its G blocks and
a per-monomer pass sums them in pair order, so a solve repeats bitwise, a batch
cluster equals its solo solve bitwise, and the results stay within rounding
of the default (atomic) accumulation and within 1e-10 of the oracle."""
import json
import os

import numpy as np
import pytest

from synth import make_cluster_batch, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def bitwise(a, b):
    return np.array_equal(np.asarray(a).view(np.uint64), np.asarray(b).view(np.uint64))


@pytest.mark.parametrize("prec", [mc.MCPT_FP64, mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp64", "fp32polish", "bf16polish"])
def test_repeats_bitwise_and_matches_oracle(ctx, prec):
    with open(os.path.join(GOLDEN, "hf-5x5x5-c2.json")) as f:
        g = json.load(f)
    pid = ctx.upload(make_workload("hf-5x5x5-c2"))
    runs = []
    for _ in range(3):
        s = ctx.run(pid, tol=1e-10, precision=prec, polish=1, deterministic=1)
        runs.append((s, ctx.energy(pid)))
    ref_s, ref_e = runs[0]
    for s, e in runs[1:]:
        assert s["e_total"] == ref_s["e_total"] and s["sweeps"] == ref_s["sweeps"]
        for k in ("e_m2", "de_m2", "e_d2", "t"):
            assert bitwise(e[k], ref_e[k]), k
    assert abs(ref_s["e_total"] - g["e_total"]) <= 1e-10 * abs(g["e_total"])
    s_atomic = ctx.run(pid, tol=1e-10, precision=prec, polish=1)
    assert s_atomic["sweeps"] == ref_s["sweeps"]
    assert abs(s_atomic["e_total"] - ref_s["e_total"]) <= 1e-12 * abs(ref_s["e_total"])
    ctx.release(pid)


def test_batch_cluster_equals_solo_bitwise(ctx):
    probs = make_cluster_batch(4, min_mono=3, max_mono=14, first=500)
    pid = ctx.upload_batch(probs)
    ctx.run(pid, tol=1e-10, deterministic=1)
    per = ctx.cluster_results(pid)
    e = ctx.energy(pid)
    sl = ctx.cluster_slices(pid)
    ctx.release(pid)
    for q, p in enumerate(probs):
        sid = ctx.upload(p)
        s1 = ctx.run(sid, tol=1e-10, deterministic=1)
        e1 = ctx.energy(sid)
        ctx.release(sid)
        assert per[q]["sweeps"] == s1["sweeps"]
        assert per[q]["e_total"] == s1["e_total"], q
        ms, ps = sl[q]
        assert bitwise(e["e_m2"][ms], e1["e_m2"]) and bitwise(e["e_d2"][ps], e1["e_d2"])


@pytest.mark.parametrize("prec", [mc.MCPT_FP64, mc.MCPT_FP32], ids=["fp64", "fp32polish"])
def test_graph_replay_bitwise_equal_to_eager(ctx, prec):
    pid = ctx.upload(make_workload("hf-2x2x2"))
    a = ctx.run(pid, tol=1e-10, precision=prec, polish=1, deterministic=1)
    ea = ctx.energy(pid)
    for _ in range(2):
        b = ctx.run(pid, tol=1e-10, precision=prec, polish=1, deterministic=1, graph=1, check_every=2)
        eb = ctx.energy(pid)
        assert b["e_total"] == a["e_total"] and b["sweeps"] == a["sweeps"]
        assert bitwise(eb["t"], ea["t"])
    ctx.release(pid)


def test_partials_count_against_the_budget():
    prob = make_workload("hf-5x5x5-c2")
    with mc.Context(0, hbm_budget=2 * prob.nbytes() + (64 << 20)) as small:   # solve fits, partials do not
        pid = small.upload(prob)
        assert small.run(pid, tol=1e-10)["status"] == mc.MCPT_OK
        with pytest.raises(mc.MCPTError) as ei:
            small.run(pid, tol=1e-10, deterministic=1)
        assert ei.value.status == mc.MCPT_ERR_ADMISSION
