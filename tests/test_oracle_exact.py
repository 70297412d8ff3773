"""Pins of the oracle's exact and truncated layers against closed forms (CPU only)."""

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import exact, trunc
from workloads import simple_cubic


@pytest.fixture(scope="module")
def sc8():
    H = simple_cubic(8)
    return H, H.to_dense()


def test_exact_matches_simple_cubic_band(sc8):
    H, Hd = sc8
    for T, mu in [(0.1, 0.0), (0.3, 0.7), (0.05, -1.2)]:
        ex = exact.observables(Hd, T, mu)
        cl = cf.observables(8, -1.0, T, mu)
        for key in ("N", "E", "F", "S"):
            assert abs(ex[key] - cl[key]) <= 1e-12 * max(1.0, abs(cl[key])), key


def test_half_filling_by_particle_hole_symmetry(sc8):
    # bipartite lattice, zero onsite, mu = 0: N = n and every diagonal density entry is 1
    H, Hd = sc8
    ex = exact.observables(Hd, 0.1, 0.0)
    assert abs(ex["N"] - 512.0) < 1e-10
    assert np.max(np.abs(np.diag(ex["P"]) - 1.0)) < 1e-12


def test_density_entries_match_plane_wave_sum(sc8):
    H, Hd = sc8
    T, mu = 0.1, 0.4
    ex = exact.observables(Hd, T, mu)
    L = 8
    index_of = H.meta["index_of"]
    site = lambda x, y, z: int(index_of[(x % L) + L * (y % L) + L * L * (z % L)])
    for d in [(0, 0, 0), (1, 0, 0), (0, 1, 0), (1, 1, 0), (2, 1, 3), (4, 4, 4)]:
        want = cf.density_entry(L, -1.0, T, mu, d)
        for origin in [(0, 0, 0), (3, 5, 2)]:
            i = site(*origin)
            j = site(origin[0] + d[0], origin[1] + d[1], origin[2] + d[2])
            assert abs(ex["P"][i, j] - want) < 1e-13


def test_thermodynamic_derivatives():
    rng = np.random.default_rng(11)
    A = rng.standard_normal((40, 40))
    Hd = 0.5 * (A + A.T)
    T, mu, h = 0.4, 0.2, 1e-5
    ex = exact.observables(Hd, T, mu, want_matrices=False)
    dF_dmu = (exact.observables(Hd, T, mu + h, False)["F"] - exact.observables(Hd, T, mu - h, False)["F"]) / (2 * h)
    dF_dT = (exact.observables(Hd, T + h, mu, False)["F"] - exact.observables(Hd, T - h, mu, False)["F"]) / (2 * h)
    assert abs(dF_dmu + ex["N"]) < 1e-7
    assert abs(dF_dT + ex["S"]) < 1e-7
    assert abs(ex["F"] - (ex["E"] - mu * ex["N"] - T * ex["S"])) < 1e-10


def test_exact_density_is_gradient_of_free_energy():
    rng = np.random.default_rng(12)
    A = rng.standard_normal((12, 12))
    Hd = 0.5 * (A + A.T)
    T, mu, h = 0.5, 0.1, 1e-6
    P = exact.observables(Hd, T, mu)["P"]
    for (i, j) in [(0, 0), (2, 5), (7, 3), (11, 11)]:
        dH = np.zeros_like(Hd)
        dH[i, j] += 1.0
        dH[j, i] += 1.0 if i != j else 0.0
        fd = (exact.observables(Hd + h * dH, T, mu, False)["F"]
              - exact.observables(Hd - h * dH, T, mu, False)["F"]) / (2 * h)
        want = P[i, j] * (2.0 if i != j else 1.0)
        assert abs(fd - want) < 1e-7


def test_truncation_error_only(sc8):
    # truncated series differ from the exact band only by the truncation error
    # of ~exp(-6.4 p T/(e_max - e_min)) = exp(-13.5) at these settings
    H, Hd = sc8
    tr = trunc.observables(Hd, H.e_min, H.e_max, 0.1, 0.0, 256)
    cl = cf.truncated_observables(8, -1.0, H.e_min, H.e_max, 0.1, 0.0, 256)
    ex = cf.observables(8, -1.0, 0.1, 0.0)
    for key in ("N", "E", "F"):
        assert abs(tr[key] - cl[key]) < 1e-10
        assert abs(tr[key] - ex[key]) < 512 * 2e-5


def test_odd_moments_vanish_on_bipartite_lattice(sc8):
    H, Hd = sc8
    m = trunc.exact_moments(Hd, H.e_min, H.e_max, 64)
    assert abs(m[0] - 512.0) < 1e-10
    assert np.max(np.abs(m[1::2])) < 1e-9
    assert np.max(np.abs(m[2::2])) > 1.0


def test_truncated_gradient_matches_finite_difference():
    rng = np.random.default_rng(13)
    A = rng.standard_normal((16, 16))
    Hd = 0.5 * (A + A.T)
    a, b, T, mu, p, h = -8.0, 8.0, 0.6, 0.2, 60, 1e-6
    G = trunc.observables(Hd, a, b, T, mu, p)["dFdH"]
    for (i, j) in [(0, 0), (1, 4), (9, 2), (15, 15)]:
        dH = np.zeros_like(Hd)
        dH[i, j] += 1.0
        if i != j:
            dH[j, i] += 1.0
        fd = (trunc.observables(Hd + h * dH, a, b, T, mu, p, False)["F"]
              - trunc.observables(Hd - h * dH, a, b, T, mu, p, False)["F"]) / (2 * h)
        want = G[i, j] * (2.0 if i != j else 1.0)
        assert abs(fd - want) < 1e-7
