"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This package builds the Fock and overlap matrices of a model cluster of atoms
carrying normalised s-type Gaussians, and nothing else: it holds none of the
density-matrix arithmetic.  Random numbers that the method itself draws
(Rademacher probe vectors) are produced here and passed in as inputs to both
the oracle and the HIP path.
"""
from .clusters import (  # noqa: F401
    EXPONENTS,
    SPACING,
    Cluster,
    WORKLOADS,
    basis_functions,
    batch_cluster_sizes,
    cube_sites,
    grid_around,
    make_batch,
    make_cluster,
    rademacher,
    s_gaussian_pair_integrals,
    sphere_sites,
    workload,
)
