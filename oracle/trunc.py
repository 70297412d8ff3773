"""Observables with the Fermi functions replaced by their truncated Chebyshev series.

Evaluated in the eigenbasis, so that truncation error (Polynomial approximation)
is separated from sampling error (Random approximation):
  x_i = (2 eps_i - e_min - e_max)/(e_max - e_min)
  N_p = sum_i sum_k alpha^f_k T_k(x_i),  E_p likewise with alpha^{ef},  F_p with beta^g
  P_p = V diag(sum_k alpha^f_k T_k(x_i)) V^T
  dF_p/dH = (2/(e_max - e_min)) V diag(sum_k beta^g_k k U_{k-1}(x_i)) V^T
The last line is the derivative of the truncated free energy with the
interval held fixed (chain rule through the spectral map).

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import fermi as fm
from .exact import diagonalize


def mapped(eps, e_min, e_max):
    return (2.0 * np.asarray(eps) - e_min - e_max) / (e_max - e_min)


def observables(H_dense, e_min, e_max, T, mu, n_terms, want_matrices=True):
    eps, V = diagonalize(H_dense)
    x = mapped(eps, e_min, e_max)
    af, aef, bg = fm.fermi_coefficient_sets(e_min, e_max, T, mu, n_terms)
    f_p = fm.chebyshev_series(af, x)
    ef_p = fm.chebyshev_series(aef, x)
    g_p = fm.chebyshev_series(bg, x)
    out = {"eigenvalues": eps, "x": x, "N": float(f_p.sum()), "E": float(ef_p.sum()),
           "F": float(g_p.sum()), "coefficients": (af, aef, bg)}
    if want_matrices:
        out["P"] = (V * f_p) @ V.T
        dg = fm.chebyshev_series_derivative(bg, x)
        out["dFdH"] = (2.0 / (e_max - e_min)) * ((V * dg) @ V.T)
    return out


def exact_moments(H_dense, e_min, e_max, n_terms):
    """tr T_k(H_hat) for k < n_terms, from eigenvalues and T_k(cos t) = cos(k t)."""
    eps, _ = diagonalize(H_dense)
    theta = np.arccos(np.clip(mapped(eps, e_min, e_max), -1.0, 1.0))
    k = np.arange(n_terms, dtype=np.float64)
    return np.cos(np.multiply.outer(k, theta)).sum(axis=1)
