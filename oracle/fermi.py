"""Fermi-Dirac, energy-weighted and free-energy functions and their Chebyshev coefficients.

Follows the paper's Methods section (definition of the free-energy function g and
the spin-degenerate Fermi function f = g') and the Polynomial approximation
subsection (projection of the mapped function onto Chebyshev polynomials under
their orthogonality weight, evaluated by Chebyshev-Gauss quadrature).

Test infrastructure only (see the package docstring).
"""

import numpy as np
import scipy.fft


def fermi(x, T, mu):
    """f(x) = 2 / (1 + exp((x - mu)/T)), written as 1 - tanh((x - mu)/(2T)) to avoid overflow."""
    return 1.0 - np.tanh((np.asarray(x, dtype=np.float64) - mu) / (2.0 * T))


def energy_weight(x, T, mu):
    """x f(x): the function whose trace is the band energy E = tr[Q] (S = I)."""
    x = np.asarray(x, dtype=np.float64)
    return x * fermi(x, T, mu)


def free_energy(x, T, mu):
    """g(x) = -2T ln(1 + exp(-(x - mu)/T)) = -2T softplus(-(x - mu)/T), evaluated stably."""
    z = -(np.asarray(x, dtype=np.float64) - mu) / T
    softplus = np.maximum(z, 0.0) + np.log1p(np.exp(-np.abs(z)))
    return -2.0 * T * softplus


def entropy(x, T, mu):
    """Per-level entropy -2[phi ln phi + (1 - phi) ln(1 - phi)], phi = f/2 (used by the thermodynamic pin)."""
    u = (np.asarray(x, dtype=np.float64) - mu) / T
    phi = 0.5 * fermi(x, T, mu)
    # phi ln phi + (1-phi) ln(1-phi) = -ln(1+e^u) + (1-phi) u, with ln(1+e^u) = softplus(u)
    sp = np.maximum(u, 0.0) + np.log1p(np.exp(-np.abs(u)))
    return -2.0 * (-sp + (1.0 - phi) * u)


def to_energy(x, e_min, e_max):
    """Inverse spectral map: x in [-1, 1] -> e_min (1 - x)/2 + e_max (1 + x)/2."""
    return 0.5 * e_min * (1.0 - x) + 0.5 * e_max * (1.0 + x)


def chebyshev_coefficients(h, e_min, e_max, n_terms, n_nodes=None):
    """Coefficients c_k, k < n_terms, of h(e(x)) ~ sum_k c_k T_k(x) on [-1, 1].

    c_k = (2 - delta_k0)/pi * int T_k(x) h(e(x)) dx / sqrt(1 - x^2), evaluated with the
    n_nodes-point Chebyshev-Gauss rule at x_j = cos(pi (j + 1/2)/n_nodes):
        c_k = (2 - delta_k0)/n_nodes * sum_j h(e(x_j)) cos(pi k (j + 1/2)/n_nodes).
    The node sum is a type-II discrete cosine transform (library FFT).  Default
    n_nodes = 4 n_terms.
    """
    if n_nodes is None:
        n_nodes = 4 * n_terms
    if n_nodes < n_terms:
        raise ValueError("need at least as many quadrature nodes as terms")
    j = np.arange(n_nodes, dtype=np.float64)
    x = np.cos(np.pi * (j + 0.5) / n_nodes)
    vals = np.asarray(h(to_energy(x, e_min, e_max)), dtype=np.float64)
    # scipy's DCT-II: y_k = 2 sum_j v_j cos(pi k (2j+1) / (2 N))
    y = scipy.fft.dct(vals, type=2)
    c = y[:n_terms] / n_nodes
    c[0] *= 0.5
    return c


def fermi_coefficient_sets(e_min, e_max, T, mu, n_terms, n_nodes=None):
    """(alpha_f, alpha_ef, beta_g): coefficient sets for N, E and F."""
    af = chebyshev_coefficients(lambda e: fermi(e, T, mu), e_min, e_max, n_terms, n_nodes)
    aef = chebyshev_coefficients(lambda e: energy_weight(e, T, mu), e_min, e_max, n_terms, n_nodes)
    bg = chebyshev_coefficients(lambda e: free_energy(e, T, mu), e_min, e_max, n_terms, n_nodes)
    return af, aef, bg


def chebyshev_series(c, x):
    """sum_k c_k T_k(x) with T_k(x) = cos(k arccos x), for |x| <= 1 (direct definition)."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    theta = np.arccos(x)
    k = np.arange(len(c), dtype=np.float64)
    return np.cos(np.multiply.outer(theta, k)) @ np.asarray(c)


def chebyshev_series_derivative(c, x):
    """d/dx sum_k c_k T_k(x) = sum_k c_k k U_{k-1}(x), U_{k-1}(cos t) = sin(k t)/sin(t), for |x| < 1."""
    x = np.asarray(x, dtype=np.float64)
    theta = np.arccos(np.clip(x, -1.0, 1.0))
    k = np.arange(len(c), dtype=np.float64)
    s = np.sin(theta)
    kt = np.multiply.outer(theta, k)
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.sin(kt) / s[..., None]
    # at x = +-1 use the limit U_{k-1}(+-1) = (+-1)^{k-1} k
    edge = np.abs(s) < 1e-12
    if np.any(edge):
        sign = np.sign(x[edge])[:, None]
        u[edge] = (sign ** (k - 1)) * k
    return (u * k) @ np.asarray(c)
