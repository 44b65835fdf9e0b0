"""Finite-displacement workflow on the GPU (Sec. IV.A): displaced geometries
built on the device from a resident base problem (mcpt_upload_scaled) equal
host-built ones, and the five-point second derivatives of the unit-cell energy
of Eq. 66 (mcpt_fd_stencil, warm-started displaced solves) match the oracle:
unit energies within 1e-10 relative (the FP64 bar), second derivatives within
1e-6 relative (the energies converge to 1e-12; the stencil divides their
differences by 12 h^2 = 1.2e-3 A^2, and oracle runs at tolerances 1e-12 and
1e-13 differ by ~1e-9 relative)."""
import json
import os

import numpy as np
import pytest

from oracle import mcpt_fd
from synth import (central_cell, lccd_integrals, make_lattice_problem, cubic_sites, make_workload,
                   scaled_problem, singles_source, stretch_modes)
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
E_TOL = 1e-10
D2_TOL = 1e-6
SOLVE_TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def rel(a, b):
    a, b = np.asarray(a, dtype=np.float64), np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)) if b.size else 0.0


def test_upload_scaled_equals_host_scaled(ctx):
    p = make_workload("hf-2x2x2")
    _, pairs, f = stretch_modes(p)[1]
    base = ctx.upload(p)
    dev = ctx.upload_scaled(base, pairs, f[3])
    host = ctx.upload(scaled_problem(p, pairs, f[3]))
    a = ctx.run(dev, tol=SOLVE_TOL)
    ea = ctx.energy(dev)
    b = ctx.run(host, tol=SOLVE_TOL)
    eb = ctx.energy(host)
    for pid in (dev, host, base):
        ctx.release(pid)
    assert a["sweeps"] == b["sweeps"]
    assert rel(ea["e_m2"], eb["e_m2"]) <= 1e-14 and rel(ea["e_d2"], eb["e_d2"]) <= 1e-14


@pytest.mark.parametrize("singles", [False, True])
def test_stencil_matches_oracle_small(ctx, singles):
    p = make_workload("hf-2x2x2")
    cell = central_cell(p)
    modes = stretch_modes(p, cell)
    w = singles_source(p) if singles else None
    print(f"[gpu] fd stencil hf-2x2x2 singles={singles}", flush=True)
    ref = mcpt_fd.stencil(p, [(a, f) for _, a, f in modes], cell, 0.01, tol=SOLVE_TOL, w=w)
    base = ctx.upload(p)
    out = ctx.fd_stencil(base, [(a, f) for _, a, f in modes], cell, 0.01, w=w, tol=SOLVE_TOL)
    ctx.release(base)
    for r, g in zip(out, ref):
        assert r["status"] == mc.MCPT_OK
        assert rel(r["e"], g["e"]) <= E_TOL
        assert abs(r["d2e"] - g["d2e"]) <= D2_TOL * max(1.0, abs(g["d2e"]))
        # warm starts from the base amplitudes: displaced points need fewer sweeps than the base
        assert max(r["sweeps"][k] for k in (0, 1, 3, 4)) <= r["sweeps"][2]


def test_stencil_matches_stored_oracle_125(ctx):
    with open(os.path.join(GOLDEN, "fd-hf-5x5x5-c2.json")) as f:
        g = json.load(f)
    p = make_workload("hf-5x5x5-c2")
    cell = central_cell(p)
    assert list(cell) == g["cell"]
    modes = stretch_modes(p, cell, step_angstrom=g["step_angstrom"])
    print("[gpu] fd stencil hf-5x5x5-c2 (stored oracle)", flush=True)
    base = ctx.upload(p)
    out = ctx.fd_stencil(base, [(a, f) for _, a, f in modes], cell, g["step_angstrom"], w=singles_source(p),
                         tol=g["tol"])
    ctx.release(base)
    for r, m in zip(out, g["modes"]):
        assert rel(r["e"], m["e"]) <= E_TOL, m["name"]
        assert abs(r["d2e"] - m["d2e"]) <= D2_TOL * max(1.0, abs(m["d2e"])), m["name"]


def test_base_results_kept_and_errors(ctx):
    p = make_workload("hf-2x2x2")
    cell = central_cell(p)
    modes = [(a, f) for _, a, f in stretch_modes(p, cell)][:1]
    base = ctx.upload(p)
    plain = ctx.run(base, tol=SOLVE_TOL)
    e_plain = ctx.energy(base)
    ctx.fd_stencil(base, modes, cell, 0.01, tol=SOLVE_TOL)
    e_after = ctx.energy(base)
    assert rel(e_after["e_m2"], e_plain["e_m2"]) <= 1e-14 and plain["return"] == mc.MCPT_OK
    pairs, f = modes[0]
    bad_cases = [
        (lambda: ctx.upload_scaled(base, [p.n_pair], [1.0]), mc.MCPT_ERR_INVALID),
        (lambda: ctx.upload_scaled(base, [0, 0], [1.0, 1.0]), mc.MCPT_ERR_INVALID),
        (lambda: ctx.upload_scaled(base, [0], [np.nan]), mc.MCPT_ERR_NONFINITE),
        (lambda: ctx.upload_scaled(base + 10**6, [0], [1.0]), mc.MCPT_ERR_UNKNOWN_ID),
        (lambda: ctx.fd_stencil(base, modes, [p.n_mono], 0.01, tol=SOLVE_TOL), mc.MCPT_ERR_INVALID),
        (lambda: ctx.fd_stencil(base, modes, cell, 0.0, tol=SOLVE_TOL), mc.MCPT_ERR_INVALID),
        (lambda: ctx.fd_stencil(base, modes, cell, 0.01, tol=SOLVE_TOL, warm_t=np.zeros(1)), mc.MCPT_ERR_INVALID),
    ]
    for fn, want in bad_cases:
        with pytest.raises(mc.MCPTError) as ei:
            fn()
        assert ei.value.status == want
    ctx.lccd_attach(base, lccd_integrals(p))
    with pytest.raises(mc.MCPTError) as ei:
        ctx.fd_stencil(base, modes, cell, 0.01, tol=SOLVE_TOL)
    assert ei.value.status == mc.MCPT_ERR_INVALID
    ctx.release(base)


def test_degenerate_mode_and_batch_copy(ctx):
    """A mode that moves nothing (no pairs rescaled) has five equal energies and
    a zero second derivative; a scaled copy of a batch equals the host-scaled batch."""
    p = make_workload("hf-2x2x2")
    cell = central_cell(p)
    base = ctx.upload(p)
    empty = np.zeros((4, 0))
    r = ctx.fd_stencil(base, [(np.zeros(0, dtype=np.int64), empty)], cell, 0.01, tol=SOLVE_TOL)[0]
    ctx.release(base)
    assert r["status"] == mc.MCPT_OK
    assert max(r["e"]) - min(r["e"]) <= 1e-12 * abs(r["e"][2])
    assert abs(r["d2e"]) <= 1e-6
    a = make_lattice_problem(cubic_sites(2, 2, 1), None, sizes=[(2, 3), (3, 4), (2, 2), (1, 5)], workload=930,
                             coupling_scale=1.0)
    b = make_workload("hf-2x2x2")
    pairs = np.array([a.n_pair + 1, a.n_pair + 5, 2], dtype=np.int64)   # two pairs of the second cluster, one of the first
    f = np.array([1.01, 0.97, 1.03])
    pid = ctx.upload_batch([a, b])
    dev = ctx.upload_scaled(pid, pairs, f)
    host = ctx.upload_batch([scaled_problem(a, [2], [1.03]), scaled_problem(b, [1, 5], [1.01, 0.97])])
    sd = ctx.run(dev, tol=SOLVE_TOL)
    ed = ctx.energy(dev)
    sh = ctx.run(host, tol=SOLVE_TOL)
    eh = ctx.energy(host)
    for q in (dev, host, pid):
        ctx.release(q)
    assert sd["sweeps"] == sh["sweeps"]
    assert rel(ed["e_m2"], eh["e_m2"]) <= 1e-14 and rel(ed["e_d2"], eh["e_d2"]) <= 1e-14
