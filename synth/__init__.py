"""Seeded synthetic case-control genotype data.

This package is the only code shared by the CPU oracle (``oracle/``) and the
GPU path (``paper_2201_02460_amd``).  It draws inputs only: it holds none of
the scan's arithmetic (no tables, no counting, no scores).
"""
from .genotypes import (  # noqa: F401
    WORKLOADS,
    batched_specs,
    hwe_probs,
    make_case_control,
    make_workload,
    planted_penetrance,
    random_genotypes,
    served_pool_specs,
    served_requests,
)
