"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package holds no part of the exchange computation itself: it only draws
orbitals (Gaussian sums on the finite-difference grid, orthonormalised) and
names the workloads.  Both sides of every parity comparison read the arrays
it returns.
"""
from .orbitals import (  # noqa: F401
    RAGGED_BATCH,
    WORKLOADS,
    Workload,
    gaussian_orbitals,
    make_workload,
    orthonormalise_cgs2,
    random_fields,
)
from .bloch import bloch_orbitals, orthonormalise_cgs2_complex  # noqa: F401
