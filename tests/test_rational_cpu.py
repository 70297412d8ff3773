"""Host-side checks of the library's pole fit (rfo_rational_fit, Rational
approximation, Eq. rational_fit): it needs no GPU and must agree with the
oracle's independently written fit (scipy's elliptic functions there, an
arithmetic-geometric-mean evaluation in the library)."""

import numpy as np
import pytest

from oracle import rational as ra


@pytest.fixture(scope="module")
def pkg():
    return pytest.importorskip("paper_1812_05264_amd")


@pytest.mark.parametrize("n,T,mu,a,b", [(1, 0.3, 0.0, -1.0, 1.0), (8, 0.025, 0.0, -10.0, 32.0),
                                        (20, 0.1, -2.0, -6.5, 9.0), (33, 0.01, 0.3, -1.0, 1.5),
                                        (64, 1.0, 5.0, 4.0, 40.0)])
def test_library_fit_matches_oracle_fit(pkg, n, T, mu, a, b):
    lib = pkg.rational_fit(n, T, mu, a, b)
    ref = ra.contour_fit(n, T, mu, a, b)
    for k in ("poles", "res_f", "res_g"):
        assert lib[k].shape == (2 * n,)
        err = np.max(np.abs(lib[k] - ref[k]) / np.maximum(np.abs(ref[k]), 1e-300))
        assert err < 1e-11, (k, err)
    for k in ("f0", "g0", "g1"):
        assert abs(lib[k] - ref[k]) <= 1e-15 * max(1.0, abs(ref[k]))


def test_library_fit_is_accurate(pkg):
    T, mu, a, b = 0.05, 0.2, -4.0, 6.0
    fit = pkg.rational_fit(40, T, mu, a, b)
    x = np.linspace(a, b, 20001)
    f = ra.evaluate(fit, x, "f")
    assert np.max(np.abs(f - (1.0 - np.tanh((x - mu) / (2 * T))))) < 1e-10


@pytest.mark.parametrize("args", [(0, 0.1, 0.0, -1.0, 1.0), (4, 0.0, 0.0, -1.0, 1.0),
                                  (4, 0.1, 0.0, 1.0, 1.0), (4, float("nan"), 0.0, -1.0, 1.0),
                                  (2000, 0.1, 0.0, -1.0, 1.0)])
def test_library_fit_rejects_bad_arguments(pkg, args):
    with pytest.raises(pkg.RfoError):
        pkg.rational_fit(*args)
