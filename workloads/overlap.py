"""Synthetic overlap matrix S for the Cu-like clusters (nonorthogonal basis).

On H's block pattern: S_II = I_9 and, per unordered pair I < J in the pair
order of the cluster, S_IJ = sigma exp(-r_IJ / lam) G'_IJ with G' ~ N(0, 1)^{9x9}
(stream 8 of the cluster's seed sequence), S_JI = S_IJ^T.  sigma = 0.16 gives
a condition number near 4.5 (smallest eigenvalue near 0.38), in the range of
the NRL Cu overlap.  The spectral interval of the pencil (H, S) is taken from
its dense generalized eigenvalues and widened by 1% (small clusters only).
"""

import numpy as np

SIGMA = 0.16
LAMBDA_S = 1.5


def _draws(cl):
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([20181205, cl.config_id, 8])))
    return rng.standard_normal((cl.pairs.shape[0], 9, 9))


def overlap_values(cl, positions=None, sigma=SIGMA, lam=LAMBDA_S):
    """S blocks [nnzb, 9, 9] on the cluster's H pattern at the given positions."""
    pos = cl.positions if positions is None else positions
    d = pos[cl.pairs[:, 0]] - pos[cl.pairs[:, 1]]
    r = np.sqrt((d ** 2).sum(axis=1))
    upper = (sigma * np.exp(-r / lam))[:, None, None] * _draws(cl)
    vals = np.empty((cl.col_idx.shape[0], 9, 9))
    k0, k1, k2 = cl.slot_kind == 0, cl.slot_kind == 1, cl.slot_kind == 2
    vals[k0] = np.eye(9)
    vals[k1] = upper[cl.slot_src[k1]]
    vals[k2] = np.transpose(upper[cl.slot_src[k2]], (0, 2, 1))
    return vals


def overlap_torch(cl, positions, sigma=SIGMA, lam=LAMBDA_S):
    """Same as overlap_values, written with torch ops so that autograd can differentiate it."""
    import torch
    pos = positions
    pairs = torch.as_tensor(cl.pairs, device=pos.device)
    d = pos[pairs[:, 0]] - pos[pairs[:, 1]]
    r = torch.sqrt((d ** 2).sum(dim=1))
    g = torch.as_tensor(_draws(cl), device=pos.device, dtype=pos.dtype)
    upper = (sigma * torch.exp(-r / lam))[:, None, None] * g
    kind = torch.as_tensor(cl.slot_kind, device=pos.device)
    src = torch.as_tensor(cl.slot_src, device=pos.device)
    out = torch.empty((cl.col_idx.shape[0], 9, 9), device=pos.device, dtype=pos.dtype)
    out[kind == 0] = torch.eye(9, device=pos.device, dtype=pos.dtype)
    out[kind == 1] = upper[src[kind == 1]]
    out[kind == 2] = upper[src[kind == 2]].transpose(1, 2)
    return out


def dS_dR(cl, positions=None, sigma=SIGMA, lam=LAMBDA_S):
    """d S_IJ / d R_I [nnzb, 3, 9, 9] = -(1/lam) u_IJ S_IJ off the diagonal, 0 on it."""
    pos = cl.positions if positions is None else positions
    vals = overlap_values(cl, pos, sigma, lam)
    rows = np.repeat(np.arange(cl.n_atoms), np.diff(cl.row_ptr))
    cols = cl.col_idx.astype(np.int64)
    d = pos[rows] - pos[cols]
    r = np.sqrt((d ** 2).sum(axis=1))
    off = rows != cols
    u = np.zeros_like(d)
    u[off] = d[off] / r[off, None]
    return -(1.0 / lam) * u[:, :, None, None] * vals[:, None, :, :]


def pencil_interval(H, S_values, widen=0.01):
    """[e_min, e_max] around the generalized eigenvalues of (H, S), dense (small systems)."""
    import scipy.linalg as sl
    S = H.with_values(S_values).to_dense()
    ev = sl.eigh(H.to_dense(), S, eigvals_only=True)
    c, h = 0.5 * (ev[-1] + ev[0]), 0.5 * (ev[-1] - ev[0]) * (1.0 + widen)
    return c - h, c + h


def pencil_bound(H, S_values, widen=0.01):
    """A rigorous interval for the pencil (H, S) of a large system: for S-normalized
    v, |v^T H v| / v^T S v <= max|spec H| / lambda_min(S); lambda_min(S) by sparse
    Lanczos, max|spec H| from H's own interval.  Wider than the pencil's spectrum."""
    import scipy.sparse.linalg as spla
    S = H.with_values(S_values).to_scipy().tocsr()
    lam = float(spla.eigsh(S, k=1, which="SA", tol=1e-6, return_eigenvectors=False)[0])
    if not lam > 0.0:
        raise ValueError("S is not positive definite")
    r = max(abs(H.e_min), abs(H.e_max)) / (lam * (1.0 - 1e-4)) * (1.0 + widen)
    return -r, r
