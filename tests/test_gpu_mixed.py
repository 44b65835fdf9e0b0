"""Mixed-precision form (FP32 or BF16 matrix-core contractions, FP64 denominators,
residual and energies) against the FP64 oracle.

Stated bounds, relative to the oracle's converged FP64 solution:
  * with FP64 polish (defect correction to an FP64 residual < 1e-10): energies
    within 1e-10 relative (measured ~1e-14 for totals, ~1e-12 per monomer);
  * without polish, after 12 reduced-precision sweeps of the 125-monomer crystal:
    FP32 within 2e-11 relative on E_total and 2e-9 on every E_M2 (relative to the
    largest; measured 4.7e-12 and 4.4e-10), BF16 within 1.5e-5 and 8e-5 (measured
    3.1e-6 and 1.7e-5).
"""
import json
import os

import numpy as np
import pytest

from oracle import mcpt_oracle
from synth import cubic_sites, make_lattice_problem, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
POLISH_RTOL = 1e-10
NO_POLISH_RTOL = {mc.MCPT_FP32: 2e-11, mc.MCPT_BF16: 1.5e-5}
NO_POLISH_MONO_RTOL = {mc.MCPT_FP32: 2e-9, mc.MCPT_BF16: 8e-5}


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def solve(ctx, prob, **opts):
    print(f"[gpu] mixed solve {prob.meta.get('name', '')} N={prob.n_mono} P={prob.n_pair} {opts}", flush=True)
    pid = ctx.upload(prob)
    ctx.set_timing(True)
    s = ctx.run(pid, raise_on_error=False, **opts)
    t = ctx.timing()
    ctx.set_timing(False)
    e = ctx.energy(pid) if s["return"] in (mc.MCPT_OK, mc.MCPT_ERR_NOT_CONVERGED) else None
    ctx.release(pid)
    return s, e, t


@pytest.mark.parametrize("prec", [mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp32", "bf16"])
def test_polish_reaches_fp64_accuracy_125(ctx, prec):
    with open(os.path.join(GOLDEN, "hf-5x5x5-c2.json")) as f:
        g = json.load(f)
    s, e, t = solve(ctx, make_workload("hf-5x5x5-c2"), tol=1e-10, precision=prec, polish=1)
    assert s["status"] == mc.MCPT_OK
    assert s["polish_sweeps"] >= 1 and s["sweeps"] > s["polish_sweeps"]
    assert t["lowp_launches"] == s["sweeps"] - s["polish_sweeps"]
    assert abs(s["e_total"] - g["e_total"]) <= POLISH_RTOL * abs(g["e_total"])
    assert rel(e["e_m2"], g["e_m2"]) <= POLISH_RTOL
    assert rel(np.asarray(e["e_d2"])[g["pair_index"]], g["e_d2"]) <= POLISH_RTOL


@pytest.mark.parametrize("prec", [mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp32", "bf16"])
def test_polish_mixed_sizes_against_oracle(ctx, prec):
    """n = 135, 21, 448, 36, 135 with ragged tails and non-square pairs."""
    sizes = [(5, 27), (3, 7), (8, 56), (4, 9), (5, 27)]
    p = make_lattice_problem(cubic_sites(5, 1, 1), None, sizes=sizes, workload=902)
    r = mcpt_oracle.solve(p, tol=1e-13)
    s, e, _ = solve(ctx, p, tol=1e-12, precision=prec, polish=1)
    assert s["status"] == mc.MCPT_OK
    assert abs(s["e_total"] - r.e_total) <= POLISH_RTOL * abs(r.e_total)
    assert rel(e["e_m2"], r.e_m2) <= POLISH_RTOL
    assert rel(e["e_d2"], r.e_d2) <= POLISH_RTOL
    T = mc.split_t(e["t"], p.n_occ, p.n_vir)
    tmax = max(float(np.max(np.abs(t))) for t in r.T)
    assert max(float(np.max(np.abs(a - b))) for a, b in zip(T, r.T)) <= POLISH_RTOL * tmax


@pytest.mark.parametrize("prec", [mc.MCPT_FP32, mc.MCPT_BF16], ids=["fp32", "bf16"])
def test_without_polish_within_stated_bound(ctx, prec):
    with open(os.path.join(GOLDEN, "hf-5x5x5-c2.json")) as f:
        g = json.load(f)
    s, e, t = solve(ctx, make_workload("hf-5x5x5-c2"), tol=0.0, max_sweeps=12, precision=prec, polish=0)
    assert s["status"] == mc.MCPT_OK and s["sweeps"] == 12 and s["polish_sweeps"] == 0
    assert t["lowp_launches"] == 12
    err = abs(s["e_total"] - g["e_total"]) / abs(g["e_total"])
    err_m = rel(e["e_m2"], g["e_m2"])
    print(f"[gpu] no-polish precision {prec}: relative E_total error {err:.3e}, per-monomer E_M2 {err_m:.3e}",
          flush=True)
    assert err <= NO_POLISH_RTOL[prec]
    assert err_m <= NO_POLISH_MONO_RTOL[prec]


def test_polish_divergence_detected(ctx):
    s, _, _ = solve(ctx, make_workload("hf-2x2x2", coupling_scale=1.0), tol=1e-10, max_sweeps=60,
                    precision=mc.MCPT_BF16, polish=1)
    assert s["return"] == mc.MCPT_ERR_DIVERGED


def test_switching_precision_on_one_resident_problem(ctx):
    p = make_workload("hf-2x2x2")
    pid = ctx.upload(p)
    out = {}
    for prec in (mc.MCPT_BF16, mc.MCPT_FP32, mc.MCPT_FP64, mc.MCPT_BF16):
        s = ctx.run(pid, tol=1e-11, precision=prec, polish=1)
        out.setdefault(prec, []).append(s["e_total"])
    ctx.release(pid)
    ref = out[mc.MCPT_FP64][0]
    for prec, vals in out.items():
        for v in vals:
            assert abs(v - ref) <= 1e-10 * abs(ref)
