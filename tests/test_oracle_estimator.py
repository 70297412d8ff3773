"""Pins of the oracle's randomized estimator: identity probes, brute force, statistics (CPU only)."""

import numpy as np
import pytest

from oracle import estimator as est
from oracle import fermi as fm
from oracle import trunc
from workloads import BSR, cu_cluster, identity_probes, rademacher, simple_cubic


def random_sparse_symmetric(n, density, seed, e_pad=1.05):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) * (rng.random((n, n)) < density)
    A = np.triu(A, 1)
    A = A + A.T + np.diag(rng.standard_normal(n))
    rows, cols = np.nonzero(A + np.eye(n))
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    w = np.linalg.eigvalsh(A)
    half = e_pad * max(abs(w[0]), abs(w[-1]))
    return BSR(row_ptr, cols.astype(np.int32), A[rows, cols].reshape(-1, 1, 1).copy(), 1, -half, half)


@pytest.fixture(scope="module")
def sc6():
    return simple_cubic(6, disorder=0.8, config_id=7)


@pytest.fixture(scope="module")
def cu13():
    return cu_cluster(13, config_id=9).bsr()


@pytest.mark.parametrize("which", ["sc6", "cu13"])
def test_identity_probes_give_truncated_exact(which, request):
    H = request.getfixturevalue(which)
    T, mu, p = 0.3, 0.2, 96
    Hd = H.to_dense()
    tr = trunc.observables(Hd, H.e_min, H.e_max, T, mu, p)
    o = est.estimate(H, identity_probes(H.n), T, mu, p, weights=np.ones(H.n), density=True, gradient=True)
    for key in ("N", "E", "F"):
        assert abs(o[key] - tr[key]) < 1e-11 * max(1.0, abs(tr[key])), key
    # per-k trace equals the eigenvalue route tr T_k = sum_i cos(k arccos x_i)
    assert np.max(np.abs(o["moments"].sum(axis=0) - trunc.exact_moments(Hd, H.e_min, H.e_max, p))) < 1e-10
    rows, cols, bd = H.block_rows(), H.col_idx, H.block_dim
    Pp = np.stack([tr["P"][bd * r:bd * r + bd, bd * c:bd * c + bd] for r, c in zip(rows, cols)])
    Gp = np.stack([tr["dFdH"][bd * r:bd * r + bd, bd * c:bd * c + bd] for r, c in zip(rows, cols)])
    assert np.max(np.abs(o["density"] - Pp)) < 1e-12
    assert np.max(np.abs(o["dFdH"] - Gp)) < 1e-11
    assert abs(o["F_grad_pass"] - o["F"]) < 1e-10


def test_moments_match_eigenbasis_per_probe():
    H = random_sparse_symmetric(24, 0.2, 3)
    R = rademacher(24, 5, config_id=77)
    p = 40
    mu_ = est.moments(est.mapped_hamiltonian(H), R, p)
    eps, V = np.linalg.eigh(H.to_dense())
    th = np.arccos(np.clip(trunc.mapped(eps, H.e_min, H.e_max), -1, 1))
    proj = V.T @ R                                   # [n, s]
    want = np.einsum("kn,nc->ck", np.cos(np.outer(np.arange(p), th)), proj ** 2)
    assert np.max(np.abs(mu_ - want)) < 1e-12
    assert np.all(np.abs(mu_[:, 0] - 24.0) == 0.0)
    assert np.all(np.abs(mu_) <= 24.0 * (1 + 1e-12))


def _fd_single_entry(H, R, T, mu, p, nz, a, b, h=1e-6):
    def F(delta):
        v = H.values.copy()
        v[nz, a, b] += delta
        return est.estimate(H.with_values(v), R, T, mu, p)["F"]
    return (F(h) - F(-h)) / (2 * h)


@pytest.mark.parametrize("case", ["bd1", "bd9"])
def test_gradient_matches_brute_force_single_entries(case):
    # F(H) with fixed probes is a polynomial in the entries; perturbing ONE entry (not its mirror)
    # measures the raw gradient entry and so also pins its orientation
    if case == "bd1":
        H = random_sparse_symmetric(24, 0.25, 4)
        R = rademacher(24, 3, config_id=78)
        picks = [(0, 0, 0), (5, 0, 0), (17, 0, 0), (H.nnzb - 1, 0, 0)]
    else:
        H = cu_cluster(3, config_id=10).bsr()
        R = rademacher(27, 2, config_id=79)
        picks = [(0, 0, 0), (1, 2, 7), (4, 8, 1), (H.nnzb - 1, 5, 5)]
    T, mu, p = 0.7, 0.1, 48
    G = est.estimate(H, R, T, mu, p, gradient=True)["dFdH"]
    for nz, a, b in picks:
        fd = _fd_single_entry(H, R, T, mu, p, nz, a, b)
        assert abs(fd - G[nz, a, b]) < 2e-7 * max(1.0, abs(G[nz, a, b])), (nz, a, b)


def test_gradient_is_symmetric_on_the_pattern(cu13):
    H = cu13
    R = rademacher(H.n, 4, config_id=80)
    G = est.estimate(H, R, 0.3, 0.0, 64, gradient=True)["dFdH"]
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    pos = {(int(r), int(c)): z for z, (r, c) in enumerate(zip(rows, cols))}
    t = np.array([pos[(int(c), int(r))] for r, c in zip(rows, cols)])
    assert np.max(np.abs(G - np.transpose(G[t], (0, 2, 1)))) < 1e-12 * np.max(np.abs(G))


def test_density_orientation_with_unit_probe(sc6):
    # a single probe e_J: X R R^T keeps only column J of X
    H = sc6
    J = 37
    R = np.zeros((H.n, 1))
    R[J, 0] = 1.0
    T, mu, p = 0.3, 0.2, 96
    o = est.estimate(H, R, T, mu, p, weights=np.ones(1), density=True)
    Pp = trunc.observables(H.to_dense(), H.e_min, H.e_max, T, mu, p)["P"]
    rows, cols = H.block_rows(), H.col_idx
    D = o["density"][:, 0, 0]
    incol = cols == J
    assert np.max(np.abs(D[~incol])) == 0.0
    assert np.max(np.abs(D[incol] - Pp[rows[incol], J])) < 1e-13


def test_sampling_error_statistics(sc6):
    # z-scores of the electron count over 100 independent probe sets: mean 0, spread 1, with the
    # Rademacher standard error sqrt(2 sum_{i != j} P_ij^2 / s) of the truncated P
    H = sc6
    T, mu, p, s = 0.3, 0.2, 64, 8
    tr = trunc.observables(H.to_dense(), H.e_min, H.e_max, T, mu, p)
    P = tr["P"]
    off = P - np.diag(np.diag(P))
    sigma = np.sqrt(2.0 * np.sum(off ** 2) / s)
    Hhat = est.mapped_hamiltonian(H)
    af = fm.chebyshev_coefficients(lambda e: fm.fermi(e, T, mu), H.e_min, H.e_max, p)
    z = []
    for seed in range(100):
        R = rademacher(H.n, s, config_id=1000 + seed)
        m = est.moments(Hhat, R, p)
        N = est.traces(m, est.default_weights(s), (af,))[0]
        z.append((N - tr["N"]) / sigma)
    z = np.array(z)
    assert abs(z.mean()) < 0.4
    assert 0.75 < z.std() < 1.25


def test_weights_and_probe_normalisation(sc6):
    H = sc6
    R = rademacher(H.n, 6, config_id=81)
    m = est.moments(est.mapped_hamiltonian(H), R, 32)
    assert np.all(m[:, 0] == H.n)
    assert np.all(np.abs(m) <= H.n * (1 + 1e-12))


def test_doubling_identities_hold_for_oracle_vectors():
    """T_2j = 2 T_j^2 - T_0 and T_2j-1 = 2 T_j T_j-1 - T_1 (product formula of
    cos): moments rebuilt from inner products of y_j = T_j(H_hat) r equal the
    direct moments r . y_k."""
    H = simple_cubic(4, disorder=0.7, config_id=5)
    R = rademacher(H.n, 5, config_id=6)
    Hh = est.mapped_hamiltonian(H)
    p = 21
    ys = list(est.chebyshev_vectors(Hh, R, p))
    mu = est.moments(Hh, R, p)              # [s][p]
    for j in range(1, (p - 1) // 2 + 1):
        two_j = 2 * np.einsum("ic,ic->c", ys[j], ys[j]) - mu[:, 0]
        assert np.allclose(two_j, mu[:, 2 * j], rtol=0, atol=1e-11 * H.n)
        two_jm1 = 2 * np.einsum("ic,ic->c", ys[j], ys[j - 1]) - mu[:, 1]
        assert np.allclose(two_jm1, mu[:, 2 * j - 1], rtol=0, atol=1e-11 * H.n)


def test_gradient_on_selected_rows(cu13):
    """The row-restricted gradient (used for the full-size fixture): with identity probes it
    equals the truncated-series gradient (eigenbasis) on the selected block rows, and with
    Rademacher probes and unequal weights it equals the whole-pattern gradient on them."""
    H = cu13
    T, mu, p = 0.3, 0.2, 96
    Hh = est.mapped_hamiltonian(H)
    _, _, bg = fm.fermi_coefficient_sets(H.e_min, H.e_max, T, mu, p)
    tr = trunc.observables(H.to_dense(), H.e_min, H.e_max, T, mu, p)
    sel = [0, 4, 12]
    F, nz, G = est.free_energy_gradient_rows(Hh, identity_probes(H.n), np.ones(H.n), bg, p, H,
                                             H.e_min, H.e_max, sel)
    rows, cols, bd = H.block_rows(), H.col_idx, H.block_dim
    assert set(rows[nz].tolist()) == set(sel) and nz.size == np.isin(rows, sel).sum()
    want = np.stack([tr["dFdH"][bd * r:bd * r + bd, bd * c:bd * c + bd]
                     for r, c in zip(rows[nz], cols[nz])])
    assert np.max(np.abs(G - want)) < 1e-11
    assert abs(F - tr["F"]) < 1e-10 * abs(tr["F"])
    R = rademacher(H.n, 3, config_id=84)
    w = np.array([0.5, 1.0, 0.25])
    F_all, G_all = est.free_energy_gradient(Hh, R, w, bg, p, H, H.e_min, H.e_max)
    F2, nz2, G2 = est.free_energy_gradient_rows(Hh, R, w, bg, p, H, H.e_min, H.e_max, [1, 12])
    assert abs(F2 - F_all) < 1e-13 * abs(F_all)
    assert np.max(np.abs(G2 - G_all[nz2])) < 1e-13 * np.max(np.abs(G_all))
