"""Write the stored oracle results of selected clusters of the batching workload
(64 uneven cubic-lattice clusters of 27-512 monomers, o5v27 / o8v56 half and half,
cutoff 2 spacings) used by the full-batch GPU test.

Calls only oracle/ and synth/ (never the HIP path).  Usage:
    python tests/golden/make_golden_batch.py [cluster ...]
Writes tests/golden/batch-64.json: per selected cluster the oracle's status, sweep
count, residual history, totals, every E_M2 and the E_D2 of every 7th pair.  The
default selection is the largest cluster (23: 507 monomers, 6,158 pairs), the
smallest (47: 28 monomers) and two between (21: 135, 50: 89).
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import mcpt_oracle  # noqa: E402
from synth import DEFAULT_COUPLING_SCALE, cluster_batch_sizes, make_cluster_batch  # noqa: E402

TOL = 1e-10
PAIR_STRIDE = 7
N_CLUSTERS = 64
DEFAULT = [23, 47, 21, 50]


def main(which):
    path = os.path.join(HERE, f"batch-{N_CLUSTERS}.json")
    out = {"workload": f"batch of {N_CLUSTERS} clusters (make_cluster_batch)", "coupling_scale": DEFAULT_COUPLING_SCALE,
           "tol": TOL, "sizes": cluster_batch_sizes(N_CLUSTERS), "clusters": {},
           "written_by": "tests/golden/make_golden_batch.py (oracle only)"}
    if os.path.exists(path):
        with open(path) as f:
            out["clusters"] = json.load(f).get("clusters", {})
    for c in which:
        t0 = time.time()
        prob = make_cluster_batch(N_CLUSTERS, only=[c])[0]
        r = mcpt_oracle.solve(prob, tol=TOL, max_sweeps=300)
        idx = list(range(0, prob.n_pair, PAIR_STRIDE))
        out["clusters"][str(c)] = {
            "n_mono": prob.n_mono, "n_pair": prob.n_pair, "status": r.status, "sweeps": r.sweeps,
            "residuals": r.residuals, "e_total": r.e_total, "e_mono": r.e_mono, "e_dimer": r.e_dimer,
            "e_mono0": r.e_mono0, "e_m2": r.e_m2.tolist(), "pair_index": idx,
            "e_d2": [float(r.e_d2[i]) for i in idx], "oracle_seconds": time.time() - t0,
        }
        with open(path, "w") as f:
            json.dump(out, f, indent=0)
        print(f"cluster {c}: N={prob.n_mono} P={prob.n_pair} status {r.status} sweeps {r.sweeps} "
              f"E {r.e_total!r} in {time.time() - t0:.1f}s", flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or DEFAULT)
