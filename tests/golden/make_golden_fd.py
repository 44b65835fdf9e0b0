"""Write the stored oracle results of the finite-displacement workflow (five-point
second derivatives of the unit-cell energy of Eq. 66 along the four stretch
modes) used by the GPU tests.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden_fd.py hf-5x5x5-c2
writes tests/golden/fd-<name>.json: for each mode the five unit energies and
the second derivative, at step 0.01 A, doubles and singles converged to 1e-12.
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_fd  # noqa: E402
from synth import central_cell, make_workload, singles_source, stretch_modes  # noqa: E402

TOL = 1e-12
STEP = 0.01


def main(names):
    for name in names:
        t0 = time.time()
        p = make_workload(name)
        cell = central_cell(p)
        modes = stretch_modes(p, cell, step_angstrom=STEP)
        w = singles_source(p)
        res = mcpt_fd.stencil(p, [(a, f) for _, a, f in modes], cell, STEP, tol=TOL, w=w)
        out = {"workload": name, "tol": TOL, "step_angstrom": STEP, "cell": [int(c) for c in cell],
               "modes": [{"name": n, "n_pairs": int(len(a)), "e": r["e"], "d2e": r["d2e"]}
                         for (n, a, _), r in zip(modes, res)],
               "oracle_seconds": time.time() - t0,
               "written_by": "tests/golden/make_golden_fd.py (oracle only)"}
        with open(os.path.join(HERE, f"fd-{name}.json"), "w") as f:
            json.dump(out, f, indent=0)
        print(f"{name}: " + ", ".join(f"{m['name']} {m['d2e']:.9f}" for m in out["modes"]) +
              f" in {time.time() - t0:.0f}s", flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["hf-5x5x5-c2"])
