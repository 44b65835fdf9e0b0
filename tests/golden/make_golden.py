"""Write the stored oracle results used by the GPU parity tests.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden.py hf-2x2x2 hf-5x5x5-c2 hf-10x10x10-c3
Each workload writes tests/golden/<name>.json: the oracle's status, sweep count,
residual history, totals, every per-monomer E_M2 and zero-coupling E_M2, and the
per-pair E_D2 (all of them up to 2000 pairs, else every 97th pair).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_oracle  # noqa: E402
from synth import make_workload, DEFAULT_COUPLING_SCALE  # noqa: E402

TOL = 1e-10
PAIR_STRIDE = 97


def main(names):
    for name in names:
        t0 = time.time()
        prob = make_workload(name)
        r = mcpt_oracle.solve(prob, tol=TOL, max_sweeps=200)
        stride = 1 if prob.n_pair <= 2000 else PAIR_STRIDE
        idx = list(range(0, prob.n_pair, stride))
        out = {
            "workload": name,
            "coupling_scale": DEFAULT_COUPLING_SCALE,
            "tol": TOL,
            "status": r.status,
            "sweeps": r.sweeps,
            "residuals": r.residuals,
            "e_total": r.e_total,
            "e_mono": r.e_mono,
            "e_dimer": r.e_dimer,
            "e_mono0": r.e_mono0,
            "e_m2": r.e_m2.tolist(),
            "e_m2_0": r.e_m2_0.tolist(),
            "pair_index": idx,
            "e_d2": [float(r.e_d2[i]) for i in idx],
            "oracle_seconds": time.time() - t0,
            "written_by": "tests/golden/make_golden.py (oracle only)",
        }
        with open(os.path.join(HERE, f"{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: status {r.status} sweeps {r.sweeps} E {r.e_total!r} in {time.time() - t0:.1f}s",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hf-2x2x2", "hf-5x5x5-c2"])
