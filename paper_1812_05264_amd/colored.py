"""Multi-color probe ensemble (paper: Hybrid approximation, the multi-color
vector ensemble; Implementation details, Welsh-Powell coloring).

Atoms are coloured so that two atoms closer than the coloring radius never share
a colour; every atomic orbital gets its own colour as well, so q atom colours
give q * n_orb probe columns.  Column (k, o) has a random sign on orbital o of
every atom of colour k and zeros elsewhere.  With one such sample (weights 1)
the trace estimate sum_c r_c^T X r_c equals tr X plus the same-colour,
same-orbital off-diagonal elements X_ij r_i r_j, whose atoms lie beyond the
coloring radius where the density matrix has decayed.  The probes feed the
library's probe input unchanged (Engine.set_probes with weights of one).
"""

import numpy as np


def neighbour_lists(positions, r_max):
    """CSR lists (ptr, idx) of the atoms within distance < r_max of each atom."""
    from scipy.spatial import cKDTree
    pos = np.asarray(positions, dtype=np.float64)
    n = pos.shape[0]
    pairs = cKDTree(pos).query_pairs(r_max, output_type="ndarray")
    if pairs.size:
        d = np.linalg.norm(pos[pairs[:, 0]] - pos[pairs[:, 1]], axis=1)
        pairs = pairs[d < r_max]                  # strict: at distance r_max no edge
    i = np.concatenate([pairs[:, 0], pairs[:, 1]]) if pairs.size else np.zeros(0, np.int64)
    j = np.concatenate([pairs[:, 1], pairs[:, 0]]) if pairs.size else np.zeros(0, np.int64)
    order = np.lexsort((j, i))
    i, j = i[order], j[order]
    ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ptr, i + 1, 1)
    return np.cumsum(ptr), j.astype(np.int64)


def welsh_powell(positions, r_max):
    """Colours [N] (0 .. q-1) of the atoms: vertices in order of decreasing
    degree (ties by index) take the smallest colour not used by an already
    coloured neighbour."""
    ptr, idx = neighbour_lists(positions, r_max)
    n = ptr.shape[0] - 1
    deg = np.diff(ptr)
    order = np.lexsort((np.arange(n), -deg))
    colours = np.full(n, -1, dtype=np.int64)
    for a in order:
        used = colours[idx[ptr[a]:ptr[a + 1]]]
        used = used[used >= 0]
        taken = np.zeros(used.size + 1, dtype=bool)
        taken[used[used <= used.size]] = True
        colours[a] = int(np.argmin(taken))           # first free colour
    return colours


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
