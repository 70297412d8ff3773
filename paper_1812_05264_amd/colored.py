"""Multi-color probe ensemble (paper: Hybrid approximation, the multi-color
vector ensemble; Implementation details, Welsh-Powell coloring).

Atoms are coloured so that two atoms closer than the coloring radius never share
a colour; every atomic orbital gets its own colour as well, so q atom colours
give q * n_orb probe columns.  Column (k, o) has a random sign on orbital o of
every atom of colour k and zeros elsewhere.  With one such sample (weights 1)
the trace estimate sum_c r_c^T X r_c equals tr X plus the same-colour,
same-orbital off-diagonal elements X_ij r_i r_j, whose atoms lie beyond the
coloring radius where the density matrix has decayed.  The coloring and the
probe block are built by the library (rfo_color_atoms, rfo_set_colored_probes);
colored_probes builds the same block on the host, for the oracle and tests.
"""

import numpy as np


def welsh_powell(positions, r_max):
    """Colours [N] (0 .. q-1) of the atoms from the library (rfo_color_atoms): no two
    atoms closer than r_max share a colour; vertices in order of decreasing degree
    (ties by index) take the smallest colour not used by an already coloured
    neighbour."""
    from ._rfo import color_atoms
    return color_atoms(positions, r_max)


def colored_probes(colours, n_orb, signs):
    """Probe block R [N * n_orb, q * n_orb] and weights [q * n_orb] (all one).

    signs [N, n_orb] are the random +-1 phases (drawn by the caller)."""
    colours = np.asarray(colours, dtype=np.int64)
    signs = np.asarray(signs, dtype=np.float64)
    n_atoms = colours.shape[0]
    if signs.shape != (n_atoms, n_orb):
        raise ValueError("signs must be [n_atoms, n_orb]")
    q = int(colours.max()) + 1 if n_atoms else 0
    R = np.zeros((n_atoms * n_orb, q * n_orb), dtype=np.float64)
    rows = (np.arange(n_atoms)[:, None] * n_orb + np.arange(n_orb)[None, :]).reshape(-1)
    cols = (colours[:, None] * n_orb + np.arange(n_orb)[None, :]).reshape(-1)
    R[rows, cols] = signs.reshape(-1)
    return R, np.ones(q * n_orb)
