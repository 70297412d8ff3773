"""Probe blocks R [n, s] for the random resolution of identity.

Rademacher probes have entries +-1 (= 2*bit - 1 with bits from stream 1 of the
config's seed sequence); their mean R R^T / s is the identity.  Identity
probes (R = I, s = n) turn the trace estimate into the exact trace.
"""

import numpy as np


def rademacher(n: int, s: int, config_id: int = 0, stream: int = 1) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, config_id, stream])))
    bits = rng.integers(0, 2, size=(n, s), dtype=np.int8)
    return (2.0 * bits.astype(np.float64) - 1.0)


def identity_probes(n: int) -> np.ndarray:
    return np.eye(n, dtype=np.float64)


def rademacher_signs(n_atoms: int, n_orb: int, config_id: int = 0, stream: int = 5) -> np.ndarray:
    """Random +-1 phases [n_atoms, n_orb] for a structured (multi-color) probe block."""
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, config_id, stream])))
    return 2.0 * rng.integers(0, 2, size=(n_atoms, n_orb)).astype(np.float64) - 1.0
