"""Exact observables by dense diagonalization (orthogonal basis, S = I).

The plain definitions of the paper's Methods section: with H = V diag(eps) V^T,
  F = sum_i g(eps_i)                       (free energy)
  N = sum_i f(eps_i),  E = sum_i eps_i f(eps_i)   (electron count, band energy)
  P = dF/dH = V diag(f(eps)) V^T,  Q = V diag(eps f(eps)) V^T   (density matrices)
and the entropy S with F = E - mu N - T S.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import fermi as fm


def diagonalize(H_dense):
    H = np.asarray(H_dense, dtype=np.float64)
    return np.linalg.eigh(0.5 * (H + H.T))


def observables(H_dense, T, mu, want_matrices=True):
    eps, V = diagonalize(H_dense)
    f = fm.fermi(eps, T, mu)
    out = {
        "eigenvalues": eps,
        "N": float(np.sum(f)),
        "E": float(np.sum(eps * f)),
        "F": float(np.sum(fm.free_energy(eps, T, mu))),
        "S": float(np.sum(fm.entropy(eps, T, mu))),
    }
    if want_matrices:
        out["P"] = (V * f) @ V.T
        out["Q"] = (V * (eps * f)) @ V.T
    return out
