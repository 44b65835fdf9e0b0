"""Write the stored oracle results of the full monomer equation (Eq. 58 with its
intramonomer terms; isolated LCCD of step 5) used by the GPU parity tests.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden_lccd.py hf-2x2x2 hf-5x5x5-c2 hf-10x10x10-c3
Each workload writes tests/golden/lccd-<name>.json: status, sweep counts of
step 5 and step 6, the step-6 residual history, totals, every E_M2 and E_LCCD,
and per-pair E_D2 (all of them up to 2000 pairs, else every 97th pair).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_lccd  # noqa: E402
from synth import DEFAULT_COUPLING_SCALE, LCCD_K_SCALE, make_lccd_workload  # noqa: E402
from synth.hf_lattice import SIGMA_LCCD  # noqa: E402

TOL = 1e-10
PAIR_STRIDE = 97


def main(names):
    for name in names:
        t0 = time.time()
        prob, ints = make_lccd_workload(name)
        e_iso, _, st_iso, res_iso = mcpt_lccd.isolated_lccd(prob, ints, tol=TOL, max_sweeps=400)
        print(f"{name}: step 5 status {st_iso} sweeps {len(res_iso)} in {time.time() - t0:.1f}s", flush=True)
        r = mcpt_lccd.solve(prob, ints, tol=TOL, max_sweeps=400)
        stride = 1 if prob.n_pair <= 2000 else PAIR_STRIDE
        idx = list(range(0, prob.n_pair, stride))
        out = {
            "workload": name,
            "coupling_scale": DEFAULT_COUPLING_SCALE,
            "k_scale": LCCD_K_SCALE,
            "sigma_lccd": SIGMA_LCCD,
            "tol": TOL,
            "status": r.status,
            "iso_status": st_iso,
            "iso_sweeps": len(res_iso),
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
            "written_by": "tests/golden/make_golden_lccd.py (oracle only)",
        }
        with open(os.path.join(HERE, f"lccd-{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: status {r.status} sweeps {r.sweeps} E {r.e_total!r} in {time.time() - t0:.1f}s",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hf-2x2x2", "hf-5x5x5-c2"])
