"""Seeded synthetic inputs for MCPT(2) solves (shared by the tests, the oracle
callers and the benchmark; holds none of the method's arithmetic)."""
from .hf_lattice import (  # noqa: F401
    Problem, WORKLOADS, cubic_sites, cluster_sites, pair_list, make_lattice_problem,
    make_workload, make_cluster_batch, cluster_batch_sizes, make_served_request, carve_served_request, ServedStream, concat_problems, SEED_ROOT,
    singles_source, LccdIntegrals, lccd_integrals, concat_lccd, make_lccd_workload, LCCD_K_SCALE,
    central_cell, displacement_scales, stretch_modes, scaled_problem, STRETCH_PATTERNS,
    SPACING_A, DEFAULT_COUPLING_SCALE, DimerIntegrals, dimer_integrals,
    DIMER_WORKLOADS, make_dimer_workload,
)
