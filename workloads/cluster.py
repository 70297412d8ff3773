"""Cu-like fcc cluster with nine orbitals per atom (s, p, d), orthogonal basis.

Construction (stated once here, used by every consumer):
  * fcc lattice constant a (default 3.61 A), atom-centred: integer points
    (i, j, k) with i + j + k even at position (a/2)(i, j, k).  The N points
    nearest the origin are kept; ties are broken by (i^2 + j^2 + k^2, i, j, k).
  * atoms are ordered by the Morton code of their integer coordinates, so that
    atoms close in space are close in index.
  * blocks couple atoms up to the second neighbour shell (cutoff 4.0 A: the
    shells sit at a/sqrt(2) = 2.55 A and a = 3.61 A, the third at 4.42 A).
  * onsite blocks are (G + G^T)/2 with G ~ N(0,1)^{9x9}; for every unordered
    pair I < J (lexicographic order) H_IJ = exp(-r_IJ / lam) G_IJ with
    G_IJ ~ N(0,1)^{9x9}, and H_JI = H_IJ^T.  Onsite draws come first, then
    the pair draws, all from stream 3.
  * the raw matrix is mapped to eV so that its spectrum spans about 20 eV:
    with [lo, hi] its extreme eigenvalues (Lanczos), c = (lo + hi)/2 and
    h = 1.01 (hi - lo)/2, both rounded to six significant digits, the
    Hamiltonian is (H_raw - c I) * 10 / h, whose spectrum lies in [-10, 10] eV.
    c and h are frozen for a given cluster, so displaced geometries reuse them.
"""

from dataclasses import dataclass

import numpy as np

from .bsr import BSR

LAMBDA = 1.5          # decay length of the hopping envelope, Angstrom
CUTOFF = 4.0          # Angstrom
HALF_BAND = 10.0      # eV: the spectrum is mapped inside [-10, 10]
_OFFSETS = np.array(
    [(sx, sy, 0) for sx in (1, -1) for sy in (1, -1)]
    + [(sx, 0, sz) for sx in (1, -1) for sz in (1, -1)]
    + [(0, sy, sz) for sy in (1, -1) for sz in (1, -1)]
    + [(2, 0, 0), (-2, 0, 0), (0, 2, 0), (0, -2, 0), (0, 0, 2), (0, 0, -2)],
    dtype=np.int64)


def _rng(config_id: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, config_id, stream])))


def _round6(x: float) -> float:
    return float(f"{x:.6g}")


def _spread_bits(v: np.ndarray) -> np.ndarray:
    v = v.astype(np.uint64) & np.uint64(0x3FF)
    out = np.zeros_like(v)
    for b in range(10):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def fcc_sphere(n_atoms: int) -> np.ndarray:
    """Integer coordinates [n_atoms, 3] of the atom-centred fcc sphere, Morton ordered."""
    r = (3.0 * n_atoms / (2.0 * np.pi)) ** (1.0 / 3.0)
    R = int(np.ceil(r)) + 4
    g = np.arange(-R, R + 1, dtype=np.int64)
    I, J, K = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)
    pts = pts[(pts.sum(axis=1) % 2) == 0]
    d2 = (pts ** 2).sum(axis=1)
    order = np.lexsort((pts[:, 2], pts[:, 1], pts[:, 0], d2))
    sel = pts[order[:n_atoms]]
    if d2[order[n_atoms - 1]] >= R * R:
        raise RuntimeError("fcc candidate box too small")
    shifted = sel - sel.min(axis=0)
    code = (_spread_bits(shifted[:, 0]) | (_spread_bits(shifted[:, 1]) << np.uint64(1))
            | (_spread_bits(shifted[:, 2]) << np.uint64(2)))
    return sel[np.argsort(code, kind="stable")]


@dataclass
class CuCluster:
    """A Cu-like cluster with its frozen random blocks; rebuilds H at any geometry."""
    positions: np.ndarray      # [N, 3] Angstrom
    pairs: np.ndarray          # [n_pairs, 2] int64, I < J, lexicographic
    onsite_raw: np.ndarray     # [N, 9, 9] symmetric
    pair_raw: np.ndarray       # [n_pairs, 9, 9] Gaussian blocks before the envelope
    row_ptr: np.ndarray
    col_idx: np.ndarray
    slot_kind: np.ndarray      # [nnzb] 0 onsite, 1 upper (I<J) pair block, 2 lower (transposed) block
    slot_src: np.ndarray       # [nnzb] index into onsite_raw or pair_raw
    center: float
    half: float
    config_id: int
    lam: float = LAMBDA

    @property
    def n_atoms(self) -> int:
        return int(self.positions.shape[0])

    @property
    def scale(self) -> float:
        return HALF_BAND / self.half

    def _pair_geometry(self, positions: np.ndarray):
        d = positions[self.pairs[:, 0]] - positions[self.pairs[:, 1]]
        r = np.sqrt((d ** 2).sum(axis=1))
        return d, r

    def values_at(self, positions: np.ndarray) -> np.ndarray:
        """H blocks [nnzb, 9, 9] in eV at the given positions (same pattern, frozen draws)."""
        _, r = self._pair_geometry(positions)
        s = self.scale
        upper = (s * np.exp(-r / self.lam))[:, None, None] * self.pair_raw
        onsite = s * (self.onsite_raw - self.center * np.eye(9)[None])
        vals = np.empty((self.col_idx.shape[0], 9, 9))
        k0 = self.slot_kind == 0
        k1 = self.slot_kind == 1
        k2 = self.slot_kind == 2
        vals[k0] = onsite[self.slot_src[k0]]
        vals[k1] = upper[self.slot_src[k1]]
        vals[k2] = np.transpose(upper[self.slot_src[k2]], (0, 2, 1))
        return vals

    def bsr(self, positions: np.ndarray = None) -> BSR:
        pos = self.positions if positions is None else positions
        return BSR(self.row_ptr, self.col_idx, self.values_at(pos), 9,
                   -HALF_BAND, HALF_BAND,
                   meta={"model": "cu_like", "n_atoms": self.n_atoms,
                         "config_id": self.config_id, "center": self.center,
                         "half": self.half})

    def dH_dR(self, positions: np.ndarray = None) -> np.ndarray:
        """Derivative blocks [nnzb, 3, 9, 9]: d H_IJ / d R_I for every stored block (I, J).

        With H_IJ = s exp(-|R_I - R_J|/lam) G_IJ, d H_IJ / d R_I = -(1/lam) u_IJ H_IJ with
        u_IJ = (R_I - R_J)/|R_I - R_J|; onsite blocks do not depend on positions.
        """
        pos = self.positions if positions is None else positions
        vals = self.values_at(pos)
        rows = np.repeat(np.arange(self.n_atoms), np.diff(self.row_ptr))
        cols = self.col_idx.astype(np.int64)
        d = pos[rows] - pos[cols]
        r = np.sqrt((d ** 2).sum(axis=1))
        off = rows != cols
        u = np.zeros_like(d)
        u[off] = d[off] / r[off, None]
        return -(1.0 / self.lam) * u[:, :, None, None] * vals[:, None, :, :]

    def values_torch(self, positions):
        """Same as values_at, written with torch ops so that autograd can differentiate it."""
        import torch
        pos = positions
        pairs = torch.as_tensor(self.pairs, device=pos.device)
        d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
        r = torch.sqrt((d ** 2).sum(dim=1))
        s = self.scale
        pr = torch.as_tensor(self.pair_raw, device=pos.device, dtype=pos.dtype)
        upper = (s * torch.exp(-r / self.lam))[:, None, None] * pr
        ons = torch.as_tensor(s * (self.onsite_raw - self.center * np.eye(9)[None]),
                              device=pos.device, dtype=pos.dtype)
        kind = torch.as_tensor(self.slot_kind, device=pos.device)
        src = torch.as_tensor(self.slot_src, device=pos.device)
        out = torch.empty((self.col_idx.shape[0], 9, 9), device=pos.device, dtype=pos.dtype)
        out[kind == 0] = ons[src[kind == 0]]
        out[kind == 1] = upper[src[kind == 1]]
        out[kind == 2] = upper[src[kind == 2]].transpose(1, 2)
        return out


def _extreme_eigs(row_ptr, col_idx, vals, n_atoms):
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla
    A = sp.bsr_matrix((vals, col_idx, row_ptr), shape=(9 * n_atoms, 9 * n_atoms)).tocsr()
    if A.shape[0] <= 2000:
        w = np.linalg.eigvalsh(A.toarray())
        return float(w[0]), float(w[-1])
    v0 = np.ones(A.shape[0])
    lo = sla.eigsh(A, k=1, which="SA", v0=v0, tol=1e-10, return_eigenvectors=False)[0]
    hi = sla.eigsh(A, k=1, which="LA", v0=v0, tol=1e-10, return_eigenvectors=False)[0]
    return float(lo), float(hi)


def cu_cluster(n_atoms: int, config_id: int = 3, a: float = 3.61, lam: float = LAMBDA) -> CuCluster:
    ijk = fcc_sphere(n_atoms)
    positions = ijk.astype(np.float64) * (0.5 * a)
    N = n_atoms
    # neighbour search on the integer lattice: first shell |d|^2 = 2, second |d|^2 = 4
    span = int(np.abs(ijk).max()) + 3
    S = 2 * span + 1
    key = (ijk[:, 0] + span) * S * S + (ijk[:, 1] + span) * S + (ijk[:, 2] + span)
    korder = np.argsort(key)
    skey = key[korder]
    Is, Js = [], []
    for off in _OFFSETS:
        q = ijk + off
        qk = (q[:, 0] + span) * S * S + (q[:, 1] + span) * S + (q[:, 2] + span)
        pos = np.searchsorted(skey, qk)
        pos = np.minimum(pos, N - 1)
        hit = skey[pos] == qk
        J = korder[pos]
        I = np.arange(N)
        m = hit & (I < J)
        Is.append(I[m])
        Js.append(J[m])
    Is = np.concatenate(Is)
    Js = np.concatenate(Js)
    porder = np.lexsort((Js, Is))
    pairs = np.stack([Is[porder], Js[porder]], axis=1).astype(np.int64)
    dist = np.sqrt(((positions[pairs[:, 0]] - positions[pairs[:, 1]]) ** 2).sum(axis=1))
    assert np.all(dist < CUTOFF)

    rng = _rng(config_id, 3)
    g = rng.standard_normal((N, 9, 9))
    onsite_raw = 0.5 * (g + np.transpose(g, (0, 2, 1)))
    pair_raw = rng.standard_normal((pairs.shape[0], 9, 9))

    # assemble the block pattern: onsite, upper (I,J) and lower (J,I) slots
    n_pairs = pairs.shape[0]
    rows = np.concatenate([np.arange(N), pairs[:, 0], pairs[:, 1]])
    cols = np.concatenate([np.arange(N), pairs[:, 1], pairs[:, 0]])
    kind = np.concatenate([np.zeros(N, np.int8), np.ones(n_pairs, np.int8), np.full(n_pairs, 2, np.int8)])
    src = np.concatenate([np.arange(N), np.arange(n_pairs), np.arange(n_pairs)])
    o = np.lexsort((cols, rows))
    rows, cols, kind, src = rows[o], cols[o], kind[o], src[o]
    row_ptr = np.zeros(N + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)

    cl = CuCluster(positions=positions, pairs=pairs, onsite_raw=onsite_raw, pair_raw=pair_raw,
                   row_ptr=row_ptr, col_idx=cols.astype(np.int32), slot_kind=kind,
                   slot_src=src.astype(np.int64), center=0.0, half=HALF_BAND,
                   config_id=config_id, lam=lam)
    raw = cl.values_at(positions)  # center 0, scale 1: the raw matrix
    lo, hi = _extreme_eigs(row_ptr, cl.col_idx, raw, N)
    cl.center = _round6(0.5 * (lo + hi))
    cl.half = _round6(1.01 * 0.5 * (hi - lo))
    return cl


def finite_difference_atoms(row_ptr: np.ndarray, per_group: int = 16):
    """The atoms whose forces are checked by finite differences: the `per_group` atoms of
    lowest coordination (fewest stored blocks in their block row, ties by atom index) and
    the first `per_group` atoms of full coordination, by atom index."""
    coord = np.diff(np.asarray(row_ptr))
    n_at = coord.size
    low = np.lexsort((np.arange(n_at), coord))[:per_group]
    bulk = np.nonzero(coord == coord.max())[0][:per_group]
    return low.astype(np.int64), bulk.astype(np.int64)
