"""mcpt_run_static (the FP64 solve with the library's fixed Tau scratch, for
callers that cannot allocate) against mcpt_run on the same resident problems,
through the C ABI: two calls in a row, the second on a smaller problem whose
largest pair (o8v56 blocks, 448 x 448 Tau slots) limits the persistent grid to
the slots that fit.  Bar: converged solves to 1e-10 relative with equal sweep
counts, fixed sweep counts to 1e-12 (the two differ only in the order of the
pair kernels' FP64 atomics)."""
import numpy as np
import pytest

from oracle import mcpt_oracle
from synth import cubic_sites, make_lattice_problem, make_workload
import paper_1409_2700_amd as mc

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300) if a.size else 0.0


@pytest.fixture(scope="module")
def ctx():
    c = mc.Context(0)
    yield c
    c.close()


def _both(ctx, prob, rtol, **opts):
    print(f"[gpu] run / run_static N={prob.n_mono} P={prob.n_pair} {opts}", flush=True)
    pid = ctx.upload(prob)
    a = ctx.run(pid, **opts)
    ea = ctx.energy(pid)
    b = ctx.run_static(pid, **opts)
    eb = ctx.energy(pid)
    ctx.release(pid)
    assert a["sweeps"] == b["sweeps"]
    for key in ("e_total", "e_mono", "e_dimer", "e_mono0"):
        assert abs(b[key] - a[key]) <= rtol * abs(a[key]), key
    for key in ("e_m2", "e_d2", "t"):
        assert rel(eb[key], ea[key]) <= rtol, key
    return b, eb


def small_mixed():
    sizes = [(5, 27), (8, 56), (3, 17), (8, 56), (2, 9)]
    return make_lattice_problem(cubic_sites(5, 1, 1), 2, sizes=sizes, workload=951, coupling_scale=0.18)


def test_static_equals_run_then_smaller_problem(ctx):
    _both(ctx, make_workload("hf-5x5x5-c2"), 1e-10, tol=1e-10, max_sweeps=100)
    p = small_mixed()
    b, eb = _both(ctx, p, 1e-10, tol=1e-10, max_sweeps=100)
    r = mcpt_oracle.solve(p, tol=1e-10, max_sweeps=100)
    assert b["sweeps"] == r.sweeps
    assert abs(b["e_total"] - r.e_total) <= 1e-10 * abs(r.e_total)
    assert rel(eb["e_d2"], r.e_d2) <= 1e-10


def test_fixed_sweeps_repeat(ctx):
    p = small_mixed()
    for _ in range(2):
        _both(ctx, p, 1e-12, tol=0.0, max_sweeps=3)


def test_rejected_options_and_sizes(ctx):
    pid = ctx.upload(small_mixed())
    for opts in (dict(precision=mc.MCPT_FP32), dict(deterministic=1), dict(graph=1)):
        s = ctx.run_static(pid, raise_on_error=False, tol=1e-10, **opts)
        assert s["return"] == mc.MCPT_ERR_INVALID, opts
    ctx.release(pid)
    # one pair whose padded Tau slot (2944^2 doubles, 69 MB) exceeds the 64 MiB scratch
    big = make_lattice_problem(cubic_sites(2, 1, 1), None, sizes=[(6, 490), (6, 490)], workload=952,
                               coupling_scale=0.01)
    pid = ctx.upload(big)
    s = ctx.run_static(pid, raise_on_error=False, tol=1e-10)
    assert s["return"] == mc.MCPT_ERR_INVALID
    ctx.release(pid)
