"""Pins of the oracle's Fermi functions and Chebyshev coefficients (CPU only)."""

import json
import os

import numpy as np
import pytest
import scipy.special

from oracle import fermi as fm

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")


def test_polynomials_are_reproduced_exactly():
    # h(e(x)) = 0.5 T_0 + T_3 - 2 T_7 must give exactly those coefficients
    a, b = -3.0, 5.0

    def h(e):
        x = (2.0 * e - a - b) / (b - a)
        th = np.arccos(np.clip(x, -1, 1))
        return 0.5 + np.cos(3 * th) - 2.0 * np.cos(7 * th)

    c = fm.chebyshev_coefficients(h, a, b, 12)
    want = np.zeros(12)
    want[0], want[3], want[7] = 0.5, 1.0, -2.0
    assert np.max(np.abs(c - want)) < 1e-14


def test_exponential_matches_bessel_closed_form():
    # exp(x) = I_0(1) + 2 sum_k I_k(1) T_k(x)
    c = fm.chebyshev_coefficients(lambda e: np.exp(e), -1.0, 1.0, 20)
    k = np.arange(20)
    want = 2.0 * scipy.special.iv(k, 1.0)
    want[0] *= 0.5
    assert np.max(np.abs(c - want)) < 1e-15


@pytest.mark.parametrize("a,b,T,mu,p", [(-6.06, 6.06, 0.1, 0.0, 256),
                                        (-6.565, 6.565, 0.02, 0.3, 2048),
                                        (-10.0, 10.0, 0.05, 0.2, 4000)])
def test_quadrature_is_converged(a, b, T, mu, p):
    c4 = fm.chebyshev_coefficients(lambda e: fm.fermi(e, T, mu), a, b, p)
    c8 = fm.chebyshev_coefficients(lambda e: fm.fermi(e, T, mu), a, b, p, n_nodes=8 * p)
    assert np.max(np.abs(c4 - c8)) < 1e-15


def _max_error(h, a, b, p, npts=100001):
    c = fm.chebyshev_coefficients(h, a, b, p)
    x = np.linspace(-1.0, 1.0, npts)
    err = 0.0
    for lo in range(0, npts, 20000):
        xx = x[lo:lo + 20000]
        err = max(err, float(np.max(np.abs(fm.chebyshev_series(c, xx) - h(fm.to_energy(xx, a, b))))))
    return err


def test_error_decay_constant_matches_paper():
    # the paper's empirical model: error ~ exp(-6.4 p T / (e_max - e_min))
    g = json.load(open(GOLDEN))["polynomial_error_model"]
    T, a, b = 0.03, -21.0, 21.0
    h = lambda e: fm.fermi(e, T, 0.0)
    e1, e2 = _max_error(h, a, b, 1000), _max_error(h, a, b, 2000)
    rate = np.log(e1 / e2) / 1000.0 * (b - a) / T
    assert abs(rate - g["decay_constant"]) / g["decay_constant"] < 0.05


def test_paper_term_count_example():
    # p = 1470 terms reach error 1e-3 at T = 0.03 eV on a 42 eV interval; measured per spin
    # (occupation in [0, 1]); 5% fewer terms must miss the target.
    g = json.load(open(GOLDEN))["polynomial_terms_example"]
    T, half = g["T_eV"], 0.5 * g["bandwidth_eV"]
    h = lambda e: 0.5 * fm.fermi(e, T, 0.0)
    assert _max_error(h, -half, half, g["n_terms"]) <= g["max_error"]
    assert _max_error(h, -half, half, int(0.95 * g["n_terms"])) > g["max_error"]


def test_fermi_is_derivative_of_free_energy_and_symmetric():
    T, mu = 0.07, 0.3
    x = np.linspace(-2, 2, 41)
    h = 1e-5
    fd = (fm.free_energy(x + h, T, mu) - fm.free_energy(x - h, T, mu)) / (2 * h)
    assert np.max(np.abs(fd - fm.fermi(x, T, mu))) < 1e-8
    assert np.max(np.abs(fm.fermi(mu + x, T, mu) + fm.fermi(mu - x, T, mu) - 2.0)) < 1e-15
    # g = (x - mu) f - T S per level, i.e. F = E - mu N - T S
    assert np.max(np.abs(fm.free_energy(x, T, mu)
                         - ((x - mu) * fm.fermi(x, T, mu) - T * fm.entropy(x, T, mu)))) < 1e-14
    # spin-degenerate limits
    assert abs(fm.fermi(-50.0, T, mu) - 2.0) < 1e-15 and abs(fm.fermi(50.0, T, mu)) < 1e-15


def test_series_derivative_matches_finite_difference():
    rng = np.random.default_rng(5)
    c = rng.standard_normal(30) / (1 + np.arange(30)) ** 2
    x = np.linspace(-0.95, 0.95, 21)
    h = 1e-6
    fd = (fm.chebyshev_series(c, x + h) - fm.chebyshev_series(c, x - h)) / (2 * h)
    assert np.max(np.abs(fd - fm.chebyshev_series_derivative(c, x))) < 1e-7
    # endpoints use the U_{k-1}(+-1) limit
    xe = np.array([-1.0, 1.0])
    k = np.arange(30)
    want = np.array([np.sum(c * k * k * (-1.0) ** (k - 1)), np.sum(c * k * k)])
    assert np.max(np.abs(fm.chebyshev_series_derivative(c, xe) - want)) < 1e-10
