"""Pins of the nonorthogonal-basis oracle (Polynomial approximation with S,
Eq. poly_PQ; Methods) against what the mathematics fixes."""

import numpy as np

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
