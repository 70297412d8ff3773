"""Random symmetric sparse matrix with one orbital per site and uneven rows.

Used to exercise the general row layout: row lengths from 1 (an isolated site
that stores only its diagonal) up to well past one gather chunk.  Every row
stores its diagonal entry (the library requires it), zero on about 40% of the
rows.  Off-diagonal values are uniform in [-1, 1], nonzero diagonal values
uniform in [0, 1]; the interval is the union of the Gershgorin discs,
widened by 1% of its length (not centred at zero).
"""

import numpy as np

from .bsr import BSR


def random_graph(n: int, config_id: int = 0, max_extra: int = 12) -> BSR:
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, config_id, 4])))
    # each site picks 0..max_extra partners; the pattern is symmetrised
    pairs = set()
    for i in range(n):
        for j in rng.choice(n, size=int(rng.integers(0, max_extra + 1)), replace=False):
            if i != j:
                pairs.add((min(i, int(j)), max(i, int(j))))
    isolated = int(rng.integers(n))
    pairs = {(i, j) for (i, j) in pairs if isolated not in (i, j)}
    entries = {}
    for (i, j) in sorted(pairs):
        v = float(rng.uniform(-1.0, 1.0))
        entries[(i, j)] = v
        entries[(j, i)] = v
    for i in range(n):
        entries[(i, i)] = float(rng.uniform(0.0, 1.0)) if rng.random() < 0.6 else 0.0
    keys = sorted(entries)
    rows = np.array([k[0] for k in keys], dtype=np.int64)
    cols = np.array([k[1] for k in keys], dtype=np.int32)
    vals = np.array([entries[k] for k in keys], dtype=np.float64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    off = rows != cols
    radius = np.zeros(n)
    np.add.at(radius, rows[off], np.abs(vals[off]))
    diag = np.zeros(n)
    diag[rows[~off]] = vals[~off]
    lo, hi = float(np.min(diag - radius)), float(np.max(diag + radius))
    pad = 0.005 * (hi - lo)
    return BSR(row_ptr, cols, vals.reshape(-1, 1, 1), 1, lo - pad, hi + pad, {"isolated": isolated})
