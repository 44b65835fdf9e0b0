"""Write the stored singles-oracle results used by the GPU parity tests.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden_singles.py hf-2x2x2 hf-5x5x5-c2 hf-10x10x10-c3
Each workload writes tests/golden/singles-<name>.json: the singles source's
seeding (synth.singles_source of the workload), the oracle's status, sweep
count, residual history, total and first-order singles energies, every
per-monomer E_M1, and the singles amplitudes at every T_STRIDE-th element.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_singles  # noqa: E402
from synth import make_workload, singles_source, DEFAULT_COUPLING_SCALE  # noqa: E402

TOL = 1e-10
T_STRIDE = 53


def main(names):
    for name in names:
        t0 = time.time()
        prob = make_workload(name)
        w = singles_source(prob)
        r = mcpt_singles.solve(prob, w, tol=TOL, max_sweeps=500)
        t = np.concatenate([tx.ravel() for tx in r.t])
        idx = list(range(0, len(t), T_STRIDE))
        out = {
            "workload": name,
            "coupling_scale": DEFAULT_COUPLING_SCALE,
            "source": "synth.singles_source(make_workload(name))",
            "tol": TOL,
            "status": r.status,
            "sweeps": r.sweeps,
            "residuals": r.residuals,
            "e_m1_total": r.e_total,
            "e_m1_0_total": r.e_total0,
            "e_m1": r.e_m1.tolist(),
            "t_index": idx,
            "t": [float(t[i]) for i in idx],
            "oracle_seconds": time.time() - t0,
            "written_by": "tests/golden/make_golden_singles.py (oracle only)",
        }
        with open(os.path.join(HERE, f"singles-{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: status {r.status} sweeps {r.sweeps} E_M1 {r.e_total!r} in {time.time() - t0:.1f}s",
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hf-2x2x2", "hf-5x5x5-c2", "hf-10x10x10-c3"])
