"""Pins of the rational-expansion oracle (Rational approximation, Eq. rational_fit,
Eq. rational_PQ; Eq. rational_derivative with S = I) against what the
mathematics fixes: the exact Fermi-Dirac and free-energy functions, the
eigenvalues of small matrices, and finite differences."""

import numpy as np
import pytest

from oracle import exact as ex
from oracle import fermi as fm
from oracle import rational as ra
from workloads import cu_cluster, identity_probes, rademacher, simple_cubic


def max_errors(fit, T, mu, a, b, n=40001):
    x = np.linspace(a, b, n)
    ef = np.max(np.abs(ra.evaluate(fit, x, "f") - fm.fermi(x, T, mu)))
    eg = np.max(np.abs(ra.evaluate(fit, x, "g") - fm.free_energy(x, T, mu)))
    eef = np.max(np.abs(ra.evaluate(fit, x, "ef") - fm.energy_weight(x, T, mu)))
    return ef, eg, eef


@pytest.mark.parametrize("T,mu,a,b", [(0.025, 0.0, -10.0, 32.0), (0.1, -2.0, -6.5, 9.0),
                                      (0.5, 1.0, -3.0, 3.0), (0.01, 0.3, -1.0, 1.5)])
def test_fit_converges_to_fermi_and_free_energy(T, mu, a, b):
    """The approximants match f, x f and g pointwise on the whole interval, with an
    error that falls geometrically with the number of nodes."""
    errs = [max_errors(ra.contour_fit(n, T, mu, a, b), T, mu, a, b) for n in (8, 16, 32, 48)]
    ef = [e[0] for e in errs]
    assert all(ef[i + 1] < 0.2 * ef[i] or ef[i + 1] < 1e-13 for i in range(len(ef) - 1)), ef
    assert ef[-1] < 1e-11
    scale = max(abs(a - mu), abs(b - mu))
    assert errs[-1][1] < 1e-9 * scale            # g grows linearly with |x - mu|
    assert errs[-1][2] < 1e-10 * scale


def test_fit_structure():
    fit = ra.contour_fit(12, 0.05, 0.4, -3.0, 5.0)
    z = fit["poles"]
    assert z.shape == (24,) and fit["res_f"].shape == (24,) and fit["res_g"].shape == (24,)
    assert np.all(z.imag > 0)
    # the first pole lies inside the band of width pi T around the real axis at
    # the left end of the contour (|xi - m| < m there), so some Im z < pi T
    assert np.min(z.imag) < np.pi * 0.05
    # mirror pairs mu + s, mu - conj(s): symmetric about Re z = mu
    n = 12
    assert np.allclose(z[:n] - 0.4, -np.conj(z[n:] - 0.4), atol=1e-14)
    # f(mu + X) + f(mu - X) = 2 is kept exactly by the fit's structure
    x = np.linspace(0.0, 3.0, 101)
    s = ra.evaluate(fit, 0.4 + x, "f") + ra.evaluate(fit, 0.4 - x, "f")
    assert np.max(np.abs(s - 2.0)) < 1e-12


def test_fit_rejects_no_nodes():
    with pytest.raises(ValueError):
        ra.contour_fit(0, 0.1, 0.0, -1.0, 1.0)


def test_jacobi_functions_at_complex_argument():
    """sn^2 + cn^2 = 1, dn^2 + m sn^2 = 1, and the values at real points and at
    i K'/2 (|sn| = 1/sqrt(k) on the line Im t = K'/2)."""
    import scipy.special as ss
    m = 0.83
    x = np.linspace(-2.0, 2.0, 9)
    y = np.full_like(x, 0.37)
    sn, cn, dn = ra.jacobi_sncndn(x, y, m)
    assert np.allclose(sn * sn + cn * cn, 1.0, atol=1e-13)
    assert np.allclose(dn * dn + m * sn * sn, 1.0, atol=1e-13)
    s0, c0, d0, _ = ss.ellipj(x, m)
    sr, cr, dr = ra.jacobi_sncndn(x, np.zeros_like(x), m)
    assert np.allclose(sr, s0, atol=1e-15) and np.allclose(cr, c0, atol=1e-15)
    Kp = ss.ellipk(1.0 - m)
    sh, _, _ = ra.jacobi_sncndn(x, np.full_like(x, 0.5 * Kp), m)
    assert np.allclose(np.abs(sh), m ** -0.25, atol=1e-12)
    # derivative d sn/dt = cn dn (complex step along the imaginary direction)
    h = 1e-6
    sp_, _, _ = ra.jacobi_sncndn(x, y + h, m)
    sm_, _, _ = ra.jacobi_sncndn(x, y - h, m)
    assert np.allclose((sp_ - sm_) / (2j * h), cn * dn, atol=1e-8)


def test_identity_probes_give_traces_of_the_fit():
    """With R = I (weights 1): N, E, F are the sums of the approximants over the
    eigenvalues, the density blocks are those of V diag(f_rat) V^T, and with an
    accurate fit they are the exact observables."""
    H = cu_cluster(13, config_id=61).bsr()
    T, mu = 0.3, 0.2
    fit = ra.contour_fit(40, T, mu, H.e_min, H.e_max)
    o = ra.estimate(H, identity_probes(H.n), fit, weights=np.ones(H.n), density=True)
    x = ra.exact(H.to_dense(), fit)
    for k in ("N", "E", "F"):
        assert abs(o[k] - x[k]) < 1e-10 * max(1.0, abs(x[k])), k
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    Pb = np.stack([x["P"][9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])
    assert np.max(np.abs(o["density"] - Pb)) < 1e-11
    e = ex.observables(H.to_dense(), T, mu)
    for k in ("N", "E", "F"):
        assert abs(o[k] - e[k]) < 1e-8 * max(1.0, abs(e[k])), k


def test_gradient_matches_finite_differences():
    """<dF/dH, dH> against central differences of the same probe estimate along
    symmetric perturbations on the block pattern."""
    H = cu_cluster(19, config_id=62).bsr()
    T, mu = 0.2, 0.1
    fit = ra.contour_fit(24, T, mu, H.e_min, H.e_max)
    R = rademacher(H.n, 5, config_id=62)
    o = ra.estimate(H, R, fit, gradient=True)
    rng = np.random.default_rng(7)
    tpos = {(int(i), int(j)): nz for nz, (i, j) in enumerate(zip(H.block_rows(), H.col_idx))}
    for _ in range(3):
        d = rng.standard_normal(H.values.shape)
        sym = np.empty_like(d)
        for (i, j), nz in tpos.items():
            sym[nz] = 0.5 * (d[nz] + d[tpos[(j, i)]].T)
        eps = 1e-5
        Fp = ra.estimate(H.with_values(H.values + eps * sym), R, fit)["F"]
        Fm = ra.estimate(H.with_values(H.values - eps * sym), R, fit)["F"]
        fd = (Fp - Fm) / (2 * eps)
        an = float(np.sum(o["dFdH"] * sym))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (fd, an)


def test_gradient_with_identity_probes_is_the_density_matrix():
    """dF/dH = P: with R = I and an accurate fit the gradient blocks are P's blocks."""
    H = simple_cubic(3, disorder=0.5, config_id=63)
    T, mu = 0.25, 0.1
    fit = ra.contour_fit(40, T, mu, H.e_min, H.e_max)
    o = ra.estimate(H, identity_probes(H.n), fit, weights=np.ones(H.n), gradient=True, density=True)
    assert np.max(np.abs(o["dFdH"] - o["density"])) < 1e-9
    P = ex.observables(H.to_dense(), T, mu)["P"]
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    assert np.max(np.abs(o["dFdH"][:, 0, 0] - P[rows, cols])) < 1e-9


def overlap_system(n_atoms, cid):
    from workloads.overlap import overlap_values, pencil_interval
    cl = cu_cluster(n_atoms, config_id=cid)
    H = cl.bsr()
    S = overlap_values(cl)
    a, b = pencil_interval(H, S)
    return H.__class__(H.row_ptr, H.col_idx, H.values, 9, a, b), S


def test_overlap_identity_reduces_to_orthogonal_estimate():
    H = cu_cluster(19, config_id=64).bsr()
    I = np.zeros_like(H.values)
    I[H.block_rows() == H.col_idx] = np.eye(9)
    R = rademacher(H.n, 6, config_id=64)
    fit = ra.contour_fit(16, 0.3, 0.1, H.e_min, H.e_max)
    o = ra.estimate_overlap(H, I, R, fit, density=True)
    e = ra.estimate(H, R, fit, density=True)
    for k in ("N", "E", "F"):
        assert abs(o[k] - e[k]) < 1e-12 * max(1.0, abs(e[k])), k
    assert np.max(np.abs(o["density"] - e["density"])) < 1e-13


def test_overlap_identity_probes_give_generalized_traces_and_P_Q():
    """With R = I and an overlap: N, E, F are the fitted functions summed over the
    generalized eigenvalues, P = V f_rat V^T and Q = V eps f_rat V^T (V^T S V = I),
    and with an accurate fit the exact generalized observables."""
    from oracle import overlap as ov
    H, S = overlap_system(13, 65)
    T, mu = 0.3, 0.2
    fit = ra.contour_fit(40, T, mu, H.e_min, H.e_max)
    o = ra.estimate_overlap(H, S, identity_probes(H.n), fit, weights=np.ones(H.n), density=True)
    Sd = H.with_values(S).to_dense()
    x = ra.exact(H.to_dense(), fit, Sd)
    for k in ("N", "E", "F"):
        assert abs(o[k] - x[k]) < 1e-10 * max(1.0, abs(x[k])), k
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    blk = lambda M: np.stack([M[9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])
    assert np.max(np.abs(o["density"] - blk(x["P"]))) < 1e-11
    assert np.max(np.abs(o["density_Q"] - blk(x["Q"]))) < 1e-10
    e = ov.exact(H.to_dense(), Sd, T, mu, H.e_min, H.e_max)
    for k in ("N", "E", "F"):
        assert abs(o[k] - e[k]) < 1e-8 * max(1.0, abs(e[k])), k


# --- the rational free-energy derivative with an overlap (Eq. rational_derivative, dS != 0) ---

def _sym_direction(H, rng):
    tpos = {(int(i), int(j)): nz for nz, (i, j) in enumerate(zip(H.block_rows(), H.col_idx))}
    d = rng.standard_normal(H.values.shape)
    sym = np.empty_like(d)
    for (i, j), nz in tpos.items():
        sym[nz] = 0.5 * (d[nz] + d[tpos[(j, i)]].T)
    return sym


def test_overlap_gradient_matches_finite_differences():
    """<dF/dH, dH> + <dF/dS, dS> against central differences of the overlap estimate along
    symmetric directions on the block pattern (H and S separately)."""
    H, S = overlap_system(13, 66)
    T, mu = 0.3, 0.2
    fit = ra.contour_fit(24, T, mu, H.e_min, H.e_max)
    R = rademacher(H.n, 4, config_id=67)
    F, GH, GS = ra.gradient_overlap(H, S, R, fit)
    assert abs(F - ra.estimate_overlap(H, S, R, fit)["F"]) < 1e-12 * abs(F)
    rng = np.random.default_rng(68)
    eps = 1e-5
    for which in ("H", "S"):
        for _ in range(2):
            d = _sym_direction(H, rng)
            if which == "H":
                Fp = ra.estimate_overlap(H.with_values(H.values + eps * d), S, R, fit)["F"]
                Fm = ra.estimate_overlap(H.with_values(H.values - eps * d), S, R, fit)["F"]
                an = float(np.sum(GH * d))
            else:
                Fp = ra.estimate_overlap(H, S + eps * d, R, fit)["F"]
                Fm = ra.estimate_overlap(H, S - eps * d, R, fit)["F"]
                an = float(np.sum(GS * d))
            fd = (Fp - Fm) / (2 * eps)
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (which, fd, an)


def test_overlap_gradient_identity_probes_closed_form():
    """R = I, weights 1: F = sum_i g_rat(eps_i) over the generalized eigenvalues, so
    dF/dH = V diag(g_rat'(eps)) V^T and dF/dS = -V diag(g_rat'(eps) eps) V^T (first-order
    perturbation of H v = eps S v, V^T S V = I), g_rat' = g1 - 2 Re sum_k tau_k/(x - z_k)^2."""
    import scipy.linalg as sl
    H, S = overlap_system(13, 69)
    T, mu = 0.3, 0.2
    fit = ra.contour_fit(20, T, mu, H.e_min, H.e_max)
    F, GH, GS = ra.gradient_overlap(H, S, identity_probes(H.n), fit, weights=np.ones(H.n))
    eps, V = sl.eigh(H.to_dense(), H.with_values(S).to_dense())
    assert abs(F - float(np.sum(ra.evaluate(fit, eps, "g")))) < 1e-10 * max(1.0, abs(F))
    gp = fit["g1"] - 2.0 * np.real((fit["res_g"][None, :] / (eps[:, None] - fit["poles"][None, :]) ** 2).sum(axis=1))
    dH = (V * gp) @ V.T
    dS = -(V * (gp * eps)) @ V.T
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    blk = lambda M: np.stack([M[9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])  # noqa: E731
    assert np.max(np.abs(GH - blk(dH))) < 1e-10 * np.max(np.abs(blk(dH)))
    assert np.max(np.abs(GS - blk(dS))) < 1e-10 * np.max(np.abs(blk(dS)))


def test_overlap_gradient_with_identity_overlap_is_the_orthogonal_one():
    H = cu_cluster(19, config_id=70).bsr()
    I = np.zeros_like(H.values)
    I[H.block_rows() == H.col_idx] = np.eye(9)
    R = rademacher(H.n, 5, config_id=70)
    fit = ra.contour_fit(16, 0.3, 0.1, H.e_min, H.e_max)
    F, GH, _ = ra.gradient_overlap(H, I, R, fit)
    e = ra.estimate(H, R, fit, gradient=True)
    assert abs(F - e["F"]) < 1e-12 * abs(e["F"])
    assert np.max(np.abs(GH - e["dFdH"])) < 1e-12 * np.max(np.abs(e["dFdH"]))
