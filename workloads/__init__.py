"""Seeded synthetic inputs shared by the HIP path, the oracle, the tests and the bench.

This package builds inputs only: block-sparse Hamiltonians of the two model
families (periodic simple-cubic orthogonal tight binding, the model proposed in
the paper's discussion section; and a Cu-like fcc cluster with nine orbitals per
atom), their derivative blocks with respect to atomic positions, and Rademacher
probe blocks.  It contains none of the Fermi-operator arithmetic (no spectral
map, Chebyshev recurrence, coefficients, traces or adjoint).

Random streams follow one convention: numpy PCG64 seeded with
``SeedSequence([20181205, config_id, stream])`` where stream 1 = probes,
2 = onsite disorder, 3 = Hamiltonian blocks.
"""

from .bsr import BSR
from .lattice import simple_cubic
from .graph import random_graph
from .cluster import CuCluster, cu_cluster, finite_difference_atoms
from .probes import rademacher, identity_probes, rademacher_signs
from .configs import CONFIGS, get_config

__all__ = [
    "BSR",
    "simple_cubic",
    "random_graph",
    "CuCluster",
    "cu_cluster",
    "finite_difference_atoms",
    "rademacher",
    "rademacher_signs",
    "identity_probes",
    "CONFIGS",
    "get_config",
]
