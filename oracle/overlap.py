"""Nonorthogonal basis (S != I), plainly: the Polynomial approximation with the
overlap and the exact generalized-eigenvalue observables (Methods).

  H_hat = [2H - (e_max + e_min) S] / (e_max - e_min)
  y_0 = y,  y_1 = H_hat S^{-1} y_0,  y_{k+1} = 2 H_hat S^{-1} y_k - y_{k-1}   (Eq. poly_PQ)
  P y ~ S^{-1} sum_k alpha^f_k y_k,   Q y ~ S^{-1} H S^{-1} sum_k alpha^f_k y_k
  N = tr[P S] (so the moments are mu_k = r . y_k as with S = I), E = tr[P H] from
  alpha^{ef}, F from beta^g, and the derivatives of that F with respect to the blocks
  of H and S (Analytical free-energy derivatives, Eq. polynomial_response).
S^{-1} is applied by a sparse LU factorization (exact up to rounding).  Exact
observables: H v = eps S v with V^T S V = I, N = sum f(eps_i), P = V f V^T,
Q = V eps f V^T; the truncated series replace f by its Chebyshev series at the
mapped eigenvalues.

Test infrastructure only (see the package docstring).
"""

import numpy as np
import scipy.linalg as sl
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fermi as fm
from .estimator import default_weights, masked_outer, traces


def mapped_pair(bsr, S_values, e_min=None, e_max=None):
    """(H_hat, S) as CSR matrices."""
    a = bsr.e_min if e_min is None else e_min
    b = bsr.e_max if e_max is None else e_max
    H = bsr.to_scipy().tocsr()
    S = bsr.with_values(S_values).to_scipy().tocsr()
    return ((2.0 * H - (a + b) * S) / (b - a)).tocsr(), S


def chebyshev_vectors(Hhat, S, R, n_terms):
    """Yields y_k = T_k(H_hat S^{-1}) R, k < n_terms."""
    lu = spla.splu(sp.csc_matrix(S))
    y_prev = np.array(R, dtype=np.float64, copy=True)
    yield y_prev
    if n_terms == 1:
        return
    y = Hhat @ lu.solve(y_prev)
    yield y
    for _ in range(2, n_terms):
        y_next = 2.0 * (Hhat @ lu.solve(y)) - y_prev
        y_prev, y = y, y_next
        yield y


def estimate(bsr, S_values, R, T, mu, n_terms, weights=None, density=False):
    """moments [s, p], N, E, F and optionally the P and Q blocks on H's pattern."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    af, aef, bg = fm.fermi_coefficient_sets(bsr.e_min, bsr.e_max, T, mu, n_terms)
    Hhat, S = mapped_pair(bsr, S_values)
    mom = np.empty((s, n_terms))
    acc = np.zeros_like(R)
    for k, y in enumerate(chebyshev_vectors(Hhat, S, R, n_terms)):
        mom[:, k] = np.einsum("ic,ic->c", R, y)
        acc += af[k] * y
    N, E, F = traces(mom, w, (af, aef, bg))
    out = {"moments": mom, "N": N, "E": E, "F": F}
    if density:
        lu = spla.splu(sp.csc_matrix(S))
        Pr = lu.solve(acc)
        Qr = lu.solve(bsr.to_scipy().tocsr() @ Pr)
        out["density"] = masked_outer(bsr, Pr, R, w)
        out["density_Q"] = masked_outer(bsr, Qr, R, w)
    return out


def _transpose_positions(bsr):
    """tpos[nz] = index of the block (J, I) for the stored block nz = (I, J)."""
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    pos = {(int(i), int(j)): z for z, (i, j) in enumerate(zip(rows, cols))}
    return np.array([pos[(int(j), int(i))] for i, j in zip(rows, cols)], dtype=np.int64)


def free_energy_gradient(bsr, S_values, R, T, mu, n_terms, weights=None):
    """(F, G_H, G_S): the probe estimate of the free energy with an overlap,
    F = sum_c w_c sum_k beta_k r_c^T T_k(A) r_c with A = H_hat S^{-1}, and its derivatives
    with respect to the blocks of H and of S, from the polynomial response (Analytical
    free-energy derivatives, Eq. polynomial_response):

      dF/dlam = sum_{j=0}^{p-2} L_j^T [dH_hat/dlam - H_hat S^{-1} dS/dlam] S^{-1} x_j,
      L_j = T_j(A^T) r   (the row vector r^T T_j(A), transposed; A^T = S^{-1} H_hat),
      x_j = (2 - delta_j0) sum_{k=j+1}^{p-1} beta_k U_{k-j-1}(A) r,

    with the spectral map dH_hat = (2 dH - (e_max + e_min) dS) / (e_max - e_min).  So on every
    stored block (I, J), with R_j = S^{-1} x_j and kappa = (e_max + e_min)/(e_max - e_min),

      G_H[I, J] = 2/(e_max - e_min) sum_j sum_c w_c L_j[I] R_j[J]^T,
      G_S[I, J] = -sum_j sum_c w_c (kappa L_j + A^T L_j)[I] R_j[J]^T,

    each returned as its symmetric part (G[I, J] + G[J, I]^T)/2, the part that symmetric
    variations of H and S (H_JI = H_IJ^T) see: with S != I the two halves differ.
    Every vector is stored; S^{-1} is a sparse LU solve."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    a, b = bsr.e_min, bsr.e_max
    p = n_terms
    _, _, bg = fm.fermi_coefficient_sets(a, b, T, mu, p)
    Hhat, S = mapped_pair(bsr, S_values)
    lu = spla.splu(sp.csc_matrix(S))
    A = lambda v: Hhat @ lu.solve(v)     # noqa: E731
    AT = lambda v: lu.solve(Hhat @ v)    # noqa: E731
    F_c = np.zeros(s)
    for k, y in enumerate(chebyshev_vectors(Hhat, S, R, p)):
        F_c += bg[k] * np.einsum("ic,ic->c", R, y)
    F = float(w @ F_c)
    nzb, bd = bsr.nnzb, bsr.block_dim
    GH = np.zeros((nzb, bd, bd))
    GS = np.zeros((nzb, bd, bd))
    if p >= 2:
        # u_m = U_m(A) r: U_0 = 1, U_1 = 2x, U_{m+1} = 2x U_m - U_{m-1}
        us = [R]
        if p > 2:
            us.append(2.0 * A(R))
        for m in range(2, p - 1):
            us.append(2.0 * A(us[m - 1]) - us[m - 2])
        # L_j = T_j(A^T) r
        Ls = [R]
        if p > 2:
            Ls.append(AT(R))
        for j in range(2, p - 1):
            Ls.append(2.0 * AT(Ls[j - 1]) - Ls[j - 2])
        kappa = (a + b) / (b - a)
        for j in range(p - 1):
            x = sum(bg[j + 1 + m] * us[m] for m in range(p - 1 - j))
            if j > 0:
                x = 2.0 * x
            Rj = lu.solve(x)
            GH += masked_outer(bsr, Ls[j], Rj, w)
            GS -= masked_outer(bsr, kappa * Ls[j] + AT(Ls[j]), Rj, w)
        GH *= 2.0 / (b - a)
    tp = _transpose_positions(bsr)
    sym = lambda G: 0.5 * (G + np.transpose(G[tp], (0, 2, 1)))   # noqa: E731
    return F, sym(GH), sym(GS)


def exact(H_dense, S_dense, T, mu, e_min, e_max, n_terms=None):
    """Generalized-eigenvalue observables; with n_terms also the truncated series."""
    eps, V = sl.eigh(H_dense, S_dense)
    f = fm.fermi(eps, T, mu)
    out = {"eigenvalues": eps, "N": float(f.sum()), "E": float((eps * f).sum()),
           "F": float(fm.free_energy(eps, T, mu).sum()),
           "P": (V * f) @ V.T, "Q": (V * (eps * f)) @ V.T}
    if n_terms:
        x = (2.0 * eps - e_min - e_max) / (e_max - e_min)
        af, aef, bg = fm.fermi_coefficient_sets(e_min, e_max, T, mu, n_terms)
        fp = fm.chebyshev_series(af, x)
        out.update({"N_p": float(fp.sum()), "E_p": float(fm.chebyshev_series(aef, x).sum()),
                    "F_p": float(fm.chebyshev_series(bg, x).sum()),
                    "P_p": (V * fp) @ V.T, "Q_p": (V * (eps * fp)) @ V.T})
    return out
