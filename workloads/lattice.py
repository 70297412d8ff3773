"""Periodic simple-cubic orthogonal tight-binding Hamiltonian (one orbital per site).

The paper's discussion section proposes clusters cut from a simple-cubic
lattice with nearest-neighbour hopping as a minimal test model.  Each row
stores its diagonal (onsite energy, possibly zero) and its six periodic
neighbours with value t, columns ascending.

Site numbering: "morton" (default) numbers the sites along a Morton
(Z-order) curve of (x, y, z), so that lattice neighbours are mostly close in
index, as for the Cu-like clusters; "natural" uses i = x + L*y + L*L*z.  The
onsite energies are drawn per lattice site in natural order, so both
numberings describe the same Hamiltonian up to a permutation.
"""

import numpy as np

from .bsr import BSR


def _rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, config_id, stream])))


def _spread3(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def site_order(L: int, ordering: str = "morton") -> np.ndarray:
    """index_of[natural site id] -> row index of that site."""
    n = L ** 3
    nat = np.arange(n, dtype=np.int64)
    if ordering == "natural":
        return nat
    if ordering != "morton":
        raise ValueError(ordering)
    x, y, z = nat % L, (nat // L) % L, nat // (L * L)
    code = _spread3(x) | (_spread3(y) << np.uint64(1)) | (_spread3(z) << np.uint64(2))
    perm = np.argsort(code, kind="stable")          # row -> natural site
    index_of = np.empty(n, dtype=np.int64)
    index_of[perm] = np.arange(n, dtype=np.int64)
    return index_of


def simple_cubic(L: int, t: float = -1.0, disorder: float = 0.0, config_id: int = 0,
                 widen: float = 0.01, ordering: str = "morton") -> BSR:
    """SC lattice L^3 with hopping t and onsite energies uniform in [-disorder/2, disorder/2].

    The returned interval is centred at 0 with half-width (1 + widen) * (6|t| + disorder/2):
    by Gershgorin's theorem the spectrum lies inside it whatever the drawn onsite values.
    """
    if L < 3:
        raise ValueError("L must be >= 3 so that the six periodic neighbours are distinct")
    n = L ** 3
    idx = np.arange(n, dtype=np.int64)          # natural site id
    x = idx % L
    y = (idx // L) % L
    z = idx // (L * L)
    nbrs = [
        ((x + 1) % L) + L * y + L * L * z,
        ((x - 1) % L) + L * y + L * L * z,
        x + L * ((y + 1) % L) + L * L * z,
        x + L * ((y - 1) % L) + L * L * z,
        x + L * y + L * L * ((z + 1) % L),
        x + L * y + L * L * ((z - 1) % L),
    ]
    index_of = site_order(L, ordering)
    cols = index_of[np.stack([idx] + nbrs, axis=1)]   # [n, 7], natural rows
    if disorder > 0.0:
        onsite = _rng(config_id, 2).uniform(-0.5 * disorder, 0.5 * disorder, size=n)
    else:
        onsite = np.zeros(n)
    vals = np.full((n, 7), float(t))
    vals[:, 0] = onsite
    # move the rows to their numbered positions
    rows_nat = np.empty(n, dtype=np.int64)
    rows_nat[index_of] = idx
    cols = cols[rows_nat]
    vals = vals[rows_nat]
    order = np.argsort(cols, axis=1, kind="stable")
    cols = np.take_along_axis(cols, order, axis=1)
    vals = np.take_along_axis(vals, order, axis=1)
    row_ptr = np.arange(0, 7 * n + 1, 7, dtype=np.int64)
    half = (1.0 + widen) * (6.0 * abs(t) + 0.5 * disorder)
    return BSR(row_ptr=row_ptr,
               col_idx=np.ascontiguousarray(cols.reshape(-1), dtype=np.int32),
               values=np.ascontiguousarray(vals.reshape(-1, 1, 1), dtype=np.float64),
               block_dim=1, e_min=-half, e_max=half,
               meta={"model": "simple_cubic", "L": L, "t": t, "disorder": disorder,
                     "config_id": config_id, "ordering": ordering, "index_of": index_of})
