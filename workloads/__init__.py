"""Seeded synthetic workloads shared by the oracle and the HIP path.

This package only *draws* problem parameters (mixture weights, means,
covariances, texture and lobe parameters, chain counts).  It holds none of
the restore method's arithmetic: no densities, no killing rates, no
estimators.  Both sides of every parity test receive exactly these
parameters and derive everything else on their own.
"""
from .generators import (  # noqa: F401
    Workload,
    gmm_iso_2d,
    gmm_iso_2d_unadjusted,
    gmm_full,
    pss_render,
    batched_uneven,
    batched_family,
    one_d_three_mode,
    WORKLOADS,
    get_workload,
)
