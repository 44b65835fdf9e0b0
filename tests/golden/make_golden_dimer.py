"""Write the stored oracle results of the full equations with the dimer-internal
terms of Eq. 59 (Tau iterated) used by the GPU parity tests and the benchmark.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden_dimer.py hf-3x3x3-c1 hf-10x10x10-c1
Each workload writes tests/golden/dimer-<name>.json: status, sweep counts of
step 5 and step 6, the step-6 residual history, totals, every E_M2 and E_LCCD,
and per-pair E_D2 (all of them up to 2000 pairs, else every 13th pair).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_dimer  # noqa: E402
from synth import DEFAULT_COUPLING_SCALE, LCCD_K_SCALE, make_dimer_workload  # noqa: E402
from synth.hf_lattice import SIGMA_DIMER, SIGMA_LCCD  # noqa: E402

TOL = 1e-10
PAIR_STRIDE = 13


def main(names):
    for name in names:
        t0 = time.time()
        prob, ints, dints = make_dimer_workload(name)
        print(f"{name}: N={prob.n_mono} P={prob.n_pair} inputs in {time.time() - t0:.1f}s", flush=True)
        r = mcpt_dimer.solve(prob, ints, dints, tol=TOL, max_sweeps=400)
        stride = 1 if prob.n_pair <= 2000 else PAIR_STRIDE
        idx = list(range(0, prob.n_pair, stride))
        out = {
            "workload": name,
            "coupling_scale": DEFAULT_COUPLING_SCALE,
            "k_scale": LCCD_K_SCALE,
            "sigma_lccd": SIGMA_LCCD,
            "sigma_dimer": SIGMA_DIMER,
            "tol": TOL,
            "status": r.status,
            "sweeps": r.sweeps,
            "residuals": r.residuals,
            "e_total": r.e_total,
            "e_mono": r.e_mono,
            "e_dimer": r.e_dimer,
            "e_lccd_total": float(sum(r.e_m2_0)),
            "e_m2": r.e_m2.tolist(),
            "e_lccd": r.e_m2_0.tolist(),
            "pair_index": idx,
            "e_d2": [float(r.e_d2[i]) for i in idx],
            "oracle_seconds": time.time() - t0,
            "written_by": "tests/golden/make_golden_dimer.py (oracle only)",
        }
        with open(os.path.join(HERE, f"dimer-{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: status {r.status} sweeps {r.sweeps} E {r.e_total!r} in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hf-3x3x3-c1", "hf-10x10x10-c1"])
