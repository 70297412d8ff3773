"""The randomized Chebyshev estimator, step by step, in FP64 with scipy sparse matrices.

Follows, in order:
  * Polynomial approximation: the spectral map
        H_hat = (2 H - (e_max + e_min) I)/(e_max - e_min)      (S = I)
    and the three-term recurrence on a probe y:
        y_0 = y,  y_1 = H_hat y_0,  y_{k+1} = 2 H_hat y_k - y_{k-1};
  * Random approximation: the estimate tr[X] ~ sum_c w_c r_c^T X r_c with the
    probes r_c as columns of R (weights w_c = 1/s for Rademacher probes, whose
    mean R R^T/s is the identity), and the random density estimator
        M (.) X_R = sum_c w_c M (.) (X r_c r_c^T);
    with X = f(H) ~ sum_k alpha_k T_k(H_hat) this is D_IJ = sum_c w_c acc_{I,c} r_{J,c}^T,
    acc_c = sum_k alpha_k y_{k,c};
  * Analytical free-energy derivatives: for F(y) = sum_j beta_j y^T T_j(H_hat) y,
        dF(y) = sum_{j=0}^{p-2} y^T T_j(H_hat) dH_hat x_j,
        x_j = (2 - delta_j0) sum_{k=j+1}^{p-1} beta_k U_{k-j-1}(H_hat) y,
    so the gradient with respect to the entries of H_hat is sum_j x_j (T_j(H_hat) y)^T,
    and dF/dH = 2/(e_max - e_min) dF/dH_hat (the interval is held fixed).

Moments are mu_{k,c} = r_c^T T_k(H_hat) r_c, returned as [s, p].

Test infrastructure only (see the package docstring).
"""

import numpy as np
import scipy.sparse as sp

from . import fermi as fm


def mapped_hamiltonian(bsr, e_min=None, e_max=None):
    """H_hat as a CSR matrix (FP64)."""
    a = bsr.e_min if e_min is None else e_min
    b = bsr.e_max if e_max is None else e_max
    H = bsr.to_scipy().tocsr().astype(np.float64)
    n = H.shape[0]
    return ((2.0 * H - (a + b) * sp.identity(n, format="csr")) / (b - a)).tocsr()


def chebyshev_vectors(Hhat, R, n_terms):
    """Yields y_0, y_1, ..., y_{n_terms-1} (each [n, s])."""
    y_prev = np.array(R, dtype=np.float64, copy=True)
    yield y_prev
    if n_terms == 1:
        return
    y = Hhat @ y_prev
    yield y
    for _ in range(2, n_terms):
        y_next = 2.0 * (Hhat @ y) - y_prev
        y_prev, y = y, y_next
        yield y


def moments(Hhat, R, n_terms):
    """mu[c, k] = r_c . y_{k,c}."""
    R = np.asarray(R, dtype=np.float64)
    out = np.empty((R.shape[1], n_terms))
    for k, y in enumerate(chebyshev_vectors(Hhat, R, n_terms)):
        out[:, k] = np.einsum("ic,ic->c", R, y)
    return out


def default_weights(s):
    return np.full(s, 1.0 / s)


def traces(mu, weights, coefficients):
    """sum_c w_c sum_k c_k mu[c, k] for each coefficient set."""
    m = np.asarray(weights) @ np.asarray(mu)          # [p]
    return [float(np.dot(c, m)) for c in coefficients]


def density_accumulator(Hhat, R, alpha, n_terms):
    """acc_c = sum_k alpha_k y_{k,c}, an estimate of f(H) r_c."""
    acc = np.zeros(np.shape(R))
    for k, y in enumerate(chebyshev_vectors(Hhat, R, n_terms)):
        acc += alpha[k] * y
    return acc


def masked_outer(bsr, X, R, weights, chunk=4096):
    """D[nz] = sum_c w_c X[I-block, c] R[J-block, c]^T for every stored block (I, J)."""
    bd = bsr.block_dim
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    s = X.shape[1]
    Xb = (np.asarray(X) * np.asarray(weights)[None, :]).reshape(-1, bd, s)
    Rb = np.asarray(R, dtype=np.float64).reshape(-1, bd, s)
    out = np.empty((bsr.nnzb, bd, bd))
    for lo in range(0, bsr.nnzb, chunk):
        hi = min(lo + chunk, bsr.nnzb)
        out[lo:hi] = np.einsum("zac,zbc->zab", Xb[rows[lo:hi]], Rb[cols[lo:hi]])
    return out


def free_energy_gradient(Hhat, R, weights, beta, n_terms, bsr, e_min, e_max):
    """(F, G): the probe estimate F = sum_c w_c sum_j beta_j r_c^T T_j(H_hat) r_c and its gradient
    G = dF/dH on the block pattern of bsr, from the U-polynomial form of the derivative
    (every y_j and every U_m(H_hat) r is stored; no checkpointing)."""
    R = np.asarray(R, dtype=np.float64)
    n, s = R.shape
    p = n_terms
    ys = np.stack(list(chebyshev_vectors(Hhat, R, p)))            # [p, n, s]
    F = float(np.dot(np.asarray(weights), np.einsum("kic,ic,k->c", ys, R, beta)))
    if p < 2:
        return F, np.zeros((bsr.nnzb, bsr.block_dim, bsr.block_dim))
    # u_m = U_m(H_hat) r:  U_0 = 1, U_1 = 2x, U_{m+1} = 2x U_m - U_{m-1}
    us = np.empty((p - 1, n, s))
    us[0] = R
    if p > 2:
        us[1] = 2.0 * (Hhat @ R)
    for m in range(2, p - 1):
        us[m] = 2.0 * (Hhat @ us[m - 1]) - us[m - 2]
    # x_j = (2 - delta_j0) sum_{m=0}^{p-2-j} beta_{j+1+m} u_m,  j = 0..p-2
    jj = np.arange(p - 1)[:, None]
    mm = np.arange(p - 1)[None, :]
    idx = jj + 1 + mm
    B = np.where(idx <= p - 1, np.asarray(beta)[np.minimum(idx, p - 1)], 0.0)
    B[1:] *= 2.0
    xs = (B @ us.reshape(p - 1, -1)).reshape(p - 1, n, s)
    # gradient on the pattern: sum_j sum_c w_c x_{j,c}[I] y_{j,c}[J]^T
    bd = bsr.block_dim
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    w = np.asarray(weights)
    Xb = (xs * w[None, None, :]).reshape(p - 1, -1, bd, s)
    Yb = ys[: p - 1].reshape(p - 1, -1, bd, s)
    G = np.empty((bsr.nnzb, bd, bd))
    chunk = max(1, 2_000_000 // max(1, (p - 1) * bd * s))
    for lo in range(0, bsr.nnzb, chunk):
        hi = min(lo + chunk, bsr.nnzb)
        G[lo:hi] = np.einsum("jzac,jzbc->zab", Xb[:, rows[lo:hi]], Yb[:, cols[lo:hi]])
    return F, (2.0 / (e_max - e_min)) * G


def estimate(bsr, R, T, mu, n_terms, weights=None, density=False, gradient=False):
    """Everything the hot path returns, computed plainly.  Keys: moments [s, p], N, E, F,
    and optionally density [nnzb, bd, bd] and dFdH [nnzb, bd, bd]."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    a, b = bsr.e_min, bsr.e_max
    Hhat = mapped_hamiltonian(bsr, a, b)
    af, aef, bg = fm.fermi_coefficient_sets(a, b, T, mu, n_terms)
    mu_ = moments(Hhat, R, n_terms)
    N, E, F = traces(mu_, w, (af, aef, bg))
    out = {"moments": mu_, "N": N, "E": E, "F": F, "weights": w,
           "coefficients": (af, aef, bg)}
    if density:
        acc = density_accumulator(Hhat, R, af, n_terms)
        out["density"] = masked_outer(bsr, acc, R, w)
    if gradient:
        F2, G = free_energy_gradient(Hhat, R, w, bg, n_terms, bsr, a, b)
        out["dFdH"] = G
        out["F_grad_pass"] = F2
    return out


def free_energy_gradient_rows(Hhat, R, weights, beta, n_terms, bsr, e_min, e_max, block_rows):
    """(F, nz, G_rows): the gradient of free_energy_gradient on the stored blocks of the given
    block rows only, for systems too large to hold every y_j and U_m(H_hat) r.

    The same U-polynomial form and the same sums: x_j = (2 - delta_j0) sum_m beta_{j+1+m} u_m
    with u_m = U_m(H_hat) r, and G_IJ = sum_j sum_c w_c x_{j,c}[I] y_{j,c}[J]^T times
    2/(e_max - e_min).  Each vector is formed whole by the recurrence; only the entries of
    the rows I (for u_m) and of their neighbour rows J (for y_j) are kept.
    nz lists the selected blocks (in pattern order), G_rows is [len(nz), bd, bd]."""
    R = np.asarray(R, dtype=np.float64)
    n, s = R.shape
    p = n_terms
    bd = bsr.block_dim
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    sel = np.isin(rows, np.asarray(block_rows, dtype=np.int64))
    nz = np.nonzero(sel)[0]
    need_I = np.unique(rows[nz])
    need_J = np.unique(cols[nz])
    oI = (need_I[:, None] * bd + np.arange(bd)[None, :]).ravel()
    oJ = (need_J[:, None] * bd + np.arange(bd)[None, :]).ravel()
    w = np.asarray(weights, dtype=np.float64)
    F_c = np.zeros(s)
    ysJ = np.empty((max(p - 1, 1), oJ.size, s))
    for k, y in enumerate(chebyshev_vectors(Hhat, R, p)):
        F_c += beta[k] * np.einsum("ic,ic->c", y, R)
        if k < p - 1:
            ysJ[k] = y[oJ]
    F = float(np.dot(w, F_c))
    if p < 2:
        return F, nz, np.zeros((nz.size, bd, bd))
    # u_m = U_m(H_hat) r:  U_0 = 1, U_1 = 2x, U_{m+1} = 2x U_m - U_{m-1}
    usI = np.empty((p - 1, oI.size, s))
    u_prev = u = None
    for m in range(p - 1):
        if m == 0:
            u_new = R
        elif m == 1:
            u_new = 2.0 * (Hhat @ R)
        else:
            u_new = 2.0 * (Hhat @ u) - u_prev
        u_prev, u = u, u_new
        usI[m] = u_new[oI]
    # x_j = (2 - delta_j0) sum_{m=0}^{p-2-j} beta_{j+1+m} u_m,  j = 0..p-2
    jj = np.arange(p - 1)[:, None]
    mm = np.arange(p - 1)[None, :]
    idx = jj + 1 + mm
    B = np.where(idx <= p - 1, np.asarray(beta)[np.minimum(idx, p - 1)], 0.0)
    B[1:] *= 2.0
    xsI = (B @ usI.reshape(p - 1, -1)).reshape(p - 1, oI.size, s)
    posI = {int(I): i for i, I in enumerate(need_I)}
    posJ = {int(J): i for i, J in enumerate(need_J)}
    G = np.empty((nz.size, bd, bd))
    for t, z in enumerate(nz):
        i0 = posI[int(rows[z])] * bd
        j0 = posJ[int(cols[z])] * bd
        X = xsI[:, i0:i0 + bd, :] * w[None, None, :]
        Y = ysJ[:, j0:j0 + bd, :]
        G[t] = np.einsum("jac,jbc->ab", X, Y)
    return F, nz, (2.0 / (e_max - e_min)) * G
