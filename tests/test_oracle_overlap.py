"""Pins of the nonorthogonal-basis oracle (Polynomial approximation with S,
Eq. poly_PQ; Methods) against what the mathematics fixes."""

import numpy as np
import pytest

from oracle import estimator as est
from oracle import overlap as ov
from workloads import cu_cluster, identity_probes, rademacher
from workloads.overlap import overlap_values, pencil_interval


def system(n_atoms, cid):
    cl = cu_cluster(n_atoms, config_id=cid)
    H = cl.bsr()
    S = overlap_values(cl)
    a, b = pencil_interval(H, S)
    return cl, H.__class__(H.row_ptr, H.col_idx, H.values, 9, a, b), S


def test_identity_overlap_reduces_to_orthogonal_estimator():
    cl = cu_cluster(19, config_id=51)
    H = cl.bsr()
    I = np.zeros_like(H.values)
    I[H.block_rows() == H.col_idx] = np.eye(9)
    R = rademacher(H.n, 7, config_id=51)
    o = ov.estimate(H, I, R, 0.3, 0.2, 50, density=True)
    e = est.estimate(H, R, 0.3, 0.2, 50, density=True)
    assert np.allclose(o["moments"], e["moments"], rtol=0, atol=1e-12 * H.n)
    for k in ("N", "E", "F"):
        assert abs(o[k] - e[k]) < 1e-12 * abs(e[k])
    assert np.allclose(o["density"], e["density"], rtol=0, atol=1e-13)


def test_identity_probes_give_truncated_generalized_traces_and_P_Q():
    """With R = I: traces are the truncated series at the generalized eigenvalues,
    S^{-1} sum alpha_k T_k(H_hat S^{-1}) = V f_p V^T and Q likewise (V^T S V = I)."""
    cl, H, S = system(13, 52)
    T, mu, p = 0.4, 0.3, 90
    o = ov.estimate(H, S, identity_probes(H.n), T, mu, p, weights=np.ones(H.n), density=True)
    x = ov.exact(H.to_dense(), H.with_values(S).to_dense(), T, mu, H.e_min, H.e_max, n_terms=p)
    for k in ("N", "E", "F"):
        assert abs(o[k] - x[k + "_p"]) < 1e-10 * max(1.0, abs(x[k + "_p"])), k
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    Pb = np.stack([x["P_p"][9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])
    Qb = np.stack([x["Q_p"][9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])
    assert np.max(np.abs(o["density"] - Pb)) < 1e-11
    assert np.max(np.abs(o["density_Q"] - Qb)) < 1e-10


def test_generalized_traces_and_truncation():
    cl, H, S = system(13, 53)
    Hd, Sd = H.to_dense(), H.with_values(S).to_dense()
    T, mu = 0.5, 0.1
    x = ov.exact(Hd, Sd, T, mu, H.e_min, H.e_max, n_terms=400)
    assert abs(np.trace(x["P"] @ Sd) - x["N"]) < 1e-10 * x["N"]     # N = tr[P S]
    assert abs(np.trace(x["P"] @ Hd) - x["E"]) < 1e-10 * max(1.0, abs(x["E"]))   # E = tr[P H]
    assert abs(x["N_p"] - x["N"]) < 1e-8 * x["N"]                   # the series converges


# --- the free-energy gradient with an overlap (Eq. polynomial_response) ----------------------

def _sym_pair(H, nz, a, b, eps):
    """Values of H plus eps on entry (a, b) of block nz and on its mirror entry, so that the
    perturbed matrix stays symmetric."""
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    I, J = int(rows[nz]), int(cols[nz])
    mirror = [z for z in range(H.nnzb) if rows[z] == J and cols[z] == I][0]
    v = np.array(H.values, copy=True)
    v[nz, a, b] += eps
    if not (mirror == nz and a == b):
        v[mirror, b, a] += eps
    return v


@pytest.mark.parametrize("which", ["H", "S"])
def test_overlap_gradient_matches_central_differences(which):
    """dF/d(entry) by central differences of the oracle's own F (fixed spectral interval),
    against 2 G_sym[I, J][a, b] for a symmetric pair of entries (G_sym[a, a] on a diagonal)."""
    cl, H, S = system(13, 55)
    R = rademacher(H.n, 3, config_id=56)
    T, mu, p = 0.5, 0.1, 30
    F0, GH, GS = ov.free_energy_gradient(H, S, R, T, mu, p)
    e = ov.estimate(H, S, R, T, mu, p)
    assert abs(F0 - e["F"]) < 1e-12 * abs(e["F"])
    G = GH if which == "H" else GS
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    rng = np.random.default_rng(57)
    picks = [int(np.nonzero(rows == cols)[0][2])] + list(rng.choice(np.nonzero(rows != cols)[0], 5,
                                                                     replace=False))
    h = 1e-4
    worst = 0.0
    for nz in picks:
        for a, b in ((0, 0), (2, 5), (7, 1)):
            if rows[nz] == cols[nz] and a == b and (a, b) != (0, 0):
                continue
            def F_at(eps):
                if which == "H":
                    return ov.estimate(H.with_values(_sym_pair(H, nz, a, b, eps)), S, R, T, mu, p)["F"]
                return ov.estimate(H, _sym_pair(H.with_values(S), nz, a, b, eps), R, T, mu, p)["F"]
            fd = (F_at(h) - F_at(-h)) / (2 * h)
            want = G[nz, a, b] if (rows[nz] == cols[nz] and a == b) else 2.0 * G[nz, a, b]
            worst = max(worst, abs(fd - want))
    scale = np.max(np.abs(G))
    print(f"{which}: worst |FD - 2 G_sym| {worst:.2e} against max |G| {scale:.2e}")
    assert worst < 1e-7 * max(1.0, scale)


def test_overlap_gradient_identity_probes_closed_form():
    """R = I, weights 1: F~ = sum_i g_p(eps_i) over the generalized eigenvalues, so
    dF~/dH = V diag(g_p'(eps)) V^T and dF~/dS = -V diag(g_p'(eps) eps) V^T (first-order
    perturbation of H v = eps S v with V^T S V = I), g_p the truncated Chebyshev series of the
    free-energy function; exact at any p."""
    cl, H, S = system(13, 58)
    T, mu, p = 0.4, 0.3, 60
    F, GH, GS = ov.free_energy_gradient(H, S, identity_probes(H.n), T, mu, p, weights=np.ones(H.n))
    Hd, Sd = H.to_dense(), H.with_values(S).to_dense()
    import scipy.linalg as sl
    from numpy.polynomial import chebyshev as C
    from oracle import fermi as fm
    eps, V = sl.eigh(Hd, Sd)
    a, b = H.e_min, H.e_max
    x = (2.0 * eps - a - b) / (b - a)
    _, _, bg = fm.fermi_coefficient_sets(a, b, T, mu, p)
    assert abs(F - float(C.chebval(x, bg).sum())) < 1e-11 * max(1.0, abs(F))
    gp = C.chebval(x, C.chebder(bg)) * 2.0 / (b - a)
    dH = (V * gp) @ V.T
    dS = -(V * (gp * eps)) @ V.T
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    blk = lambda M: np.stack([M[9 * i:9 * i + 9, 9 * j:9 * j + 9] for i, j in zip(rows, cols)])  # noqa: E731
    eH = np.max(np.abs(GH - blk(dH))) / np.max(np.abs(blk(dH)))
    eS = np.max(np.abs(GS - blk(dS))) / np.max(np.abs(blk(dS)))
    print(f"closed form: G_H {eH:.2e}, G_S {eS:.2e}")
    assert eH < 1e-10 and eS < 1e-10


def test_overlap_gradient_with_identity_overlap_is_the_orthogonal_one():
    cl = cu_cluster(19, config_id=59)
    H = cl.bsr()
    I = np.zeros_like(H.values)
    I[H.block_rows() == H.col_idx] = np.eye(9)
    R = rademacher(H.n, 5, config_id=60)
    T, mu, p = 0.3, 0.2, 40
    F, GH, _ = ov.free_energy_gradient(H, I, R, T, mu, p)
    e = est.estimate(H, R, T, mu, p, gradient=True)
    assert abs(F - e["F"]) < 1e-12 * abs(e["F"])
    assert np.max(np.abs(GH - e["dFdH"])) < 1e-12 * np.max(np.abs(e["dFdH"]))
