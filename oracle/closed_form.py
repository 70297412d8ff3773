"""Closed-form band of the periodic simple-cubic orthogonal model (onsite energy zero).

Plane waves diagonalize the nearest-neighbour hopping on an L^3 periodic
lattice: eps(k) = 2 t (cos k_x + cos k_y + cos k_z), k = 2 pi m / L.  Every
observable of the Methods section is then a k-sum, and every density-matrix
entry depends only on the displacement:
    P(d) = (1/n) sum_k f(eps(k)) cos(k . d).
This is the textbook route the paper's discussion proposes for calibrating
errors on the simple-cubic test model.

Test infrastructure only (see the package docstring).
"""

import numpy as np

from . import fermi as fm


def band(L, t=-1.0):
    k = 2.0 * np.pi * np.arange(L) / L
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    return (2.0 * t * (np.cos(kx) + np.cos(ky) + np.cos(kz))).ravel(), (kx.ravel(), ky.ravel(), kz.ravel())


def observables(L, t, T, mu):
    eps, _ = band(L, t)
    f = fm.fermi(eps, T, mu)
    return {"N": float(f.sum()), "E": float((eps * f).sum()),
            "F": float(fm.free_energy(eps, T, mu).sum()), "S": float(fm.entropy(eps, T, mu).sum())}


def density_entry(L, t, T, mu, d):
    """P between two sites separated by the integer displacement d = (dx, dy, dz)."""
    eps, (kx, ky, kz) = band(L, t)
    f = fm.fermi(eps, T, mu)
    return float(np.sum(f * np.cos(kx * d[0] + ky * d[1] + kz * d[2])) / eps.size)


def truncated_observables(L, t, e_min, e_max, T, mu, n_terms):
    """N, E, F with the truncated Chebyshev series, summed over the k-points."""
    eps, _ = band(L, t)
    x = (2.0 * eps - e_min - e_max) / (e_max - e_min)
    af, aef, bg = fm.fermi_coefficient_sets(e_min, e_max, T, mu, n_terms)
    return {"N": float(fm.chebyshev_series(af, x).sum()),
            "E": float(fm.chebyshev_series(aef, x).sum()),
            "F": float(fm.chebyshev_series(bg, x).sum())}
