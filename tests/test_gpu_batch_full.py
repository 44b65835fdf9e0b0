"""The batching workload at its full size through the C ABI: 64 uneven cubic-lattice
clusters (27-512 monomers, o5v27 / o8v56 half and half, cutoff 2 spacings; 11,253
monomers, 123,262 pairs, 83 GB of FP64 V) uploaded as one batch, every pair phase one
persistent launch per kernel variant, sweeps graph-captured, tile shape autotuned.
Selected clusters - the largest (507 monomers), the smallest (28) and two between -
are compared with stored oracle results (tests/golden/batch-64.json, oracle only):

* FP32 pair products with FP64 polish: every energy of the cluster within 1e-10
  relative (the stopping test is the FP64 residual);
* plain FP64: the same, and the cluster stops at the oracle's sweep count."""
import json
import os

import numpy as np
import pytest

from synth import make_cluster_batch
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "batch-64.json")
RTOL = 1e-10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300) if a.size else 0.0


@pytest.fixture(scope="module")
def batch():
    with open(GOLDEN) as f:
        ref = json.load(f)
    print("[gpu] generating the 64-cluster batch", flush=True)
    probs = make_cluster_batch(64, workers=min(16, os.cpu_count() or 1))
    assert [p.n_mono for p in probs] == ref["sizes"]
    ctx = mc.Context(0)
    print(f"[gpu] upload {sum(p.n_mono for p in probs)} monomers, {sum(p.n_pair for p in probs)} pairs", flush=True)
    pid = ctx.upload_batch(probs)
    yield ctx, pid, probs, ref
    ctx.release(pid)
    ctx.close()


def _compare(ctx, pid, probs, ref, fp64):
    per = ctx.cluster_results(pid)
    e = ctx.energy(pid, want_t=False)
    sl = ctx.cluster_slices(pid)
    assert all(c["status"] == mc.MCPT_OK for c in per)
    for key, g in ref["clusters"].items():
        c = int(key)
        s = per[c]
        for q in ("e_total", "e_mono", "e_dimer", "e_mono0"):
            assert abs(s[q] - g[q]) <= RTOL * abs(g[q]), (c, q, s[q], g[q])
        assert rel(e["e_m2"][sl[c][0]], g["e_m2"]) <= RTOL, c
        assert rel(e["e_d2"][sl[c][1]][g["pair_index"]], g["e_d2"]) <= RTOL, c
        if fp64:
            assert s["sweeps"] == g["sweeps"], (c, s["sweeps"], g["sweeps"])


def test_full_batch_fp32_polish_matches_oracle_clusters(batch):
    ctx, pid, probs, ref = batch
    print("[gpu] FP32 + polish, graph, autotune", flush=True)
    s = ctx.run(pid, tol=1e-10, precision=mc.MCPT_FP32, polish=1, graph=1, autotune=1)
    assert s["status"] == mc.MCPT_OK
    _compare(ctx, pid, probs, ref, fp64=False)


def test_full_batch_fp64_matches_oracle_clusters(batch):
    ctx, pid, probs, ref = batch
    print("[gpu] FP64, graph", flush=True)
    s = ctx.run(pid, tol=1e-10, precision=mc.MCPT_FP64, graph=1)
    assert s["status"] == mc.MCPT_OK
    _compare(ctx, pid, probs, ref, fp64=True)
