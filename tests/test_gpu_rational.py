"""Rational (pole) expansion on the GPU (Rational approximation, Eq. rational_fit,
Eq. rational_PQ, with and without an overlap S; Eq. rational_derivative with
S = I): CGLS on the complex-shifted systems against the oracle's sparse-LU solves
of the same fit.

Tolerance: CGLS stops at |r - (H_hat - z_hat) x| <= tol |r| per column, so the
solution error is at most kappa tol with kappa = |H_hat - z_hat| |(H_hat - z_hat)^{-1}|
<= 2 / min_k dist(z_hat_k, [-1, 1]).  The cases below keep kappa below 100;
with tol = 1e-13 every output is within 1e-11 of the exact solves, under the
1e-10 normwise bar of the other FP64 parity tests."""

import numpy as np
import pytest

from oracle import forces as ofo
from oracle import rational as ra
from tests.gpu_common import TOL, banner, check_blocks, check_rows, engine_or_skip
from workloads import BSR, cu_cluster, identity_probes, rademacher, random_graph, simple_cubic
from workloads.overlap import dS_dR, overlap_values, pencil_interval

pytestmark = pytest.mark.gpu


def fit_for(H, nodes, T, mu):
    import paper_1812_05264_amd as pkg
    return pkg.rational_fit(nodes, T, mu, H.e_min, H.e_max)


def load(eng, H, R, weights=None):
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, H.block_dim, H.e_min, H.e_max, "fp64")
    eng.set_probes(R, weights)


CASES = {
    # name: (system, s, T, mu, nodes)
    "cu55_s72": (lambda: cu_cluster(55, config_id=71), 72, 0.3, 0.2, 12),
    "sc6_s200": (lambda: simple_cubic(6, disorder=0.6, config_id=72), 200, 0.2, 0.1, 10),
    "graph300_s64": (lambda: random_graph(300, config_id=73), 64, 0.25, 0.0, 8),
    "cu13_s1000": (lambda: cu_cluster(13, config_id=74), 1000, 0.4, -0.1, 6),
}


@pytest.mark.parametrize("name", list(CASES))
def test_rational_matches_oracle(name):
    banner(f"rational parity {name}")
    make, s, T, mu, nodes = CASES[name]
    obj = make()
    H = obj.bsr() if hasattr(obj, "bsr") else obj
    R = rademacher(H.n, s, config_id=75)
    fit = fit_for(H, nodes, T, mu)
    eng = engine_or_skip()
    load(eng, H, R)
    g = eng.rational(mu, fit, tol=1e-13, max_iter=20000, density=True, gradient=True)
    o = ra.estimate(H, R, fit, density=True, gradient=True)
    for k in ("N", "E", "F"):
        assert abs(g[k] - o[k]) <= TOL * max(1.0, abs(o[k])), (k, g[k], o[k])
    check_blocks(g["density"], o["density"])
    check_blocks(g["dFdH"], o["dFdH"])
    assert g["iterations"].shape == (2 * nodes,) and np.all(g["iterations"] >= 0)
    if hasattr(obj, "dH_dR"):
        D = obj.dH_dR()
        check_rows(eng.hf_forces(D), ofo.hf_forces(H, o["dFdH"], D), what="forces")


def test_rational_identity_probes_give_traces_of_the_fit():
    """Dense (non +-1) probes R = I with unit weights: N, E, F are the traces of the
    fitted functions over the eigenvalues, and P's blocks those of V f_rat V^T."""
    banner("rational identity probes sc3")
    H = simple_cubic(3, disorder=0.4, config_id=76)
    T, mu = 0.3, 0.05
    fit = fit_for(H, 16, T, mu)
    eng = engine_or_skip()
    load(eng, H, identity_probes(H.n), np.ones(H.n))
    g = eng.rational(mu, fit, tol=1e-13, density=True)
    x = ra.exact(H.to_dense(), fit)
    for k in ("N", "E", "F"):
        assert abs(g[k] - x[k]) <= TOL * max(1.0, abs(x[k])), k
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    assert np.max(np.abs(g["density"][:, 0, 0] - x["P"][rows, cols])) < 1e-10


def test_rational_independent_of_pole_order_and_repeatable():
    """The fit's poles in reverse order (other warm starts) give the same
    observables within the solver tolerance; a repeated call is bitwise equal."""
    banner("rational order cu19")
    H = cu_cluster(19, config_id=77).bsr()
    R = rademacher(H.n, 64, config_id=77)
    fit = fit_for(H, 8, 0.3, 0.0)
    rev = {k: (v[::-1].copy() if isinstance(v, np.ndarray) else v) for k, v in fit.items()}
    eng = engine_or_skip()
    load(eng, H, R)
    a = eng.rational(0.0, fit, tol=1e-13, gradient=True)
    b = eng.rational(0.0, rev, tol=1e-13, gradient=True)
    c = eng.rational(0.0, fit, tol=1e-13, gradient=True)
    for k in ("N", "E", "F"):
        assert abs(a[k] - b[k]) <= TOL * max(1.0, abs(a[k]))
        assert a[k] == c[k]
    check_blocks(a["dFdH"], b["dFdH"])
    assert np.array_equal(a["dFdH"], c["dFdH"])
    assert np.array_equal(a["iterations"], c["iterations"])
    it, so = eng.rational_stats()
    assert so == 3 * 16 and it >= int(np.sum(a["iterations"]))


def test_rational_error_paths():
    banner("rational errors")
    import paper_1812_05264_amd as pkg
    H = simple_cubic(3, disorder=0.3, config_id=78)
    R = rademacher(H.n, 8, config_id=78)
    fit = fit_for(H, 4, 0.3, 0.0)
    eng = engine_or_skip()
    with pytest.raises(pkg.RfoError) as ei:
        eng.rational(0.0, fit)
    assert ei.value.status == "RFO_E_STATE"
    load(eng, H, R)
    bad = dict(fit, poles=np.conj(fit["poles"]))
    with pytest.raises(pkg.RfoError) as ei:
        eng.rational(0.0, bad)
    assert ei.value.status == "RFO_E_INVALID"
    for tol in (0.0, 1.0, float("nan")):
        with pytest.raises(pkg.RfoError) as ei:
            eng.rational(0.0, fit, tol=tol)
        assert ei.value.status == "RFO_E_INVALID"
    with pytest.raises(pkg.RfoError) as ei:
        eng.rational(0.0, fit, tol=1e-14, max_iter=1)
    assert ei.value.status == "RFO_E_NUMERIC"
    # the context stays usable after an error
    ok = eng.rational(0.0, fit, tol=1e-12)
    assert np.isfinite(ok["N"])
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 1, H.e_min, H.e_max, "fp32")
    eng.set_probes(R)
    with pytest.raises(pkg.RfoError) as ei:
        eng.rational(0.0, fit)
    assert ei.value.status == "RFO_E_UNSUPPORTED"


def overlap_cu(n_atoms, cid):
    cl = cu_cluster(n_atoms, config_id=cid)
    H = cl.bsr()
    S = overlap_values(cl)
    a, b = pencil_interval(H, S)
    return cl, BSR(H.row_ptr, H.col_idx, H.values, 9, a, b), S


def overlap_sc(L, cid):
    H = simple_cubic(L, disorder=0.6, config_id=cid)
    S = np.where((H.block_rows() == H.col_idx)[:, None, None], 1.0, 0.1) * np.ones_like(H.values)
    a, b = pencil_interval(H, S)
    return None, BSR(H.row_ptr, H.col_idx, H.values, 1, a, b), S


def load_overlap(eng, H, S, R, weights=None):
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, H.block_dim, H.e_min, H.e_max, "fp64")
    eng.set_overlap(S, cg_tol=1e-14)
    eng.set_probes(R, weights)


@pytest.mark.parametrize("case", ["cu43_s72", "sc6_s100", "cu13_s200"])
def test_rational_with_overlap_matches_oracle(case):
    """(H - z_k S) g_k = r: N, E, F, the P and Q blocks and the density forces
    -(tr[P dH] - tr[Q dS]) against the oracle's sparse-LU solves."""
    banner(f"rational overlap parity {case}")
    if case == "cu43_s72":
        (cl, H, S), s, T, mu, nodes = overlap_cu(43, 81), 72, 0.3, 0.2, 10
    elif case == "sc6_s100":
        (cl, H, S), s, T, mu, nodes = overlap_sc(6, 82), 100, 0.2, 0.1, 10
    else:
        (cl, H, S), s, T, mu, nodes = overlap_cu(13, 83), 200, 0.4, -0.1, 6
    R = rademacher(H.n, s, config_id=84)
    fit = fit_for(H, nodes, T, mu)
    eng = engine_or_skip()
    load_overlap(eng, H, S, R)
    g = eng.rational(mu, fit, tol=1e-13, max_iter=20000, density=True)
    Q = eng.density_q()
    o = ra.estimate_overlap(H, S, R, fit, density=True)
    for k in ("N", "E", "F"):
        assert abs(g[k] - o[k]) <= TOL * max(1.0, abs(o[k])), (k, g[k], o[k])
    check_blocks(g["density"], o["density"])
    check_blocks(Q, o["density_Q"])
    if cl is not None:
        dH, dS = cl.dH_dR(), dS_dR(cl)
        want = ofo.hf_forces(H, o["density"], dH) - ofo.hf_forces(H, o["density_Q"], dS)
        check_rows(eng.density_forces(dH, dS), want, what="density forces")
    # the same context without the overlap is the orthogonal estimate again
    eng.set_overlap(None)
    g0 = eng.rational(mu, fit, tol=1e-13, max_iter=20000)
    o0 = ra.estimate(BSR(H.row_ptr, H.col_idx, H.values, H.block_dim, H.e_min, H.e_max), R, fit)
    assert abs(g0["N"] - o0["N"]) <= TOL * abs(o0["N"])


def test_rational_with_overlap_identity_probes_give_pencil_traces():
    """R = I: N, E, F are the traces of the fitted functions over the generalized
    eigenvalues of (H, S), and the P and Q blocks those of V f V^T and V eps f V^T."""
    banner("rational overlap identity probes cu13")
    _, H, S = overlap_cu(13, 85)
    T, mu = 0.4, 0.3
    fit = fit_for(H, 14, T, mu)
    eng = engine_or_skip()
    load_overlap(eng, H, S, identity_probes(H.n), np.ones(H.n))
    g = eng.rational(mu, fit, tol=1e-13, density=True)
    Q = eng.density_q()
    x = ra.exact(H.to_dense(), fit, H.with_values(S).to_dense())
    for k in ("N", "E", "F"):
        assert abs(g[k] - x[k]) <= TOL * max(1.0, abs(x[k])), k
    rows, cols = H.block_rows(), H.col_idx.astype(np.int64)
    bd = H.block_dim
    for z in range(H.nnzb):
        blk = np.s_[rows[z] * bd:(rows[z] + 1) * bd, cols[z] * bd:(cols[z] + 1) * bd]
        assert np.max(np.abs(g["density"][z] - x["P"][blk])) < 1e-10
        assert np.max(np.abs(Q[z] - x["Q"][blk])) < 1e-10


@pytest.mark.parametrize("case", ["cu19_s72", "sc6_s100", "cu13_dense"])
def test_rational_with_overlap_gradient_matches_oracle(case):
    """dF/dH and dF/dS of the rational estimate with an overlap (Eq. rational_derivative with
    dS, and the linear part of g; two solves per pole, r and S r), as symmetric parts, against
    the oracle's sparse-LU solves; and the forces -(sum <dF/dH, dH/dR> + sum <dF/dS, dS/dR>)."""
    banner(f"rational overlap gradient {case}")
    w = None
    if case == "cu19_s72":
        (cl, H, S), s, T, mu, nodes = overlap_cu(19, 87), 72, 0.3, 0.2, 8
        R = rademacher(H.n, s, config_id=88)
    elif case == "sc6_s100":
        (cl, H, S), s, T, mu, nodes = overlap_sc(6, 89), 100, 0.2, 0.1, 8
        R = rademacher(H.n, s, config_id=90)
    else:
        (cl, H, S), s, T, mu, nodes = overlap_cu(13, 91), 37, 0.4, -0.1, 6
        R = rademacher(H.n, s, config_id=92) * (1.0 + 0.25 * np.cos(np.arange(H.n)))[:, None]
        w = np.linspace(0.5, 1.5, s) / s
    fit = fit_for(H, nodes, T, mu)
    eng = engine_or_skip()
    load_overlap(eng, H, S, R, w)
    g = eng.rational(mu, fit, tol=1e-13, max_iter=20000, gradient=True)
    GS = eng.dFdS()
    F, oH, oS = ra.gradient_overlap(H, S, R, fit, weights=w)
    assert abs(g["F"] - F) <= TOL * max(1.0, abs(F)), (g["F"], F)
    eH = check_blocks(g["dFdH"], oH, what="dF/dH")
    eS = check_blocks(GS, oS, what="dF/dS")
    print(f"{case}: dF/dH {eH:.2e}, dF/dS {eS:.2e} per block")
    if cl is not None:
        dH, dS = cl.dH_dR(), dS_dR(cl)
        want = ofo.hf_forces(H, oH, dH) + ofo.hf_forces(H, oS, dS)
        check_rows(eng.hf_forces_overlap(dH, dS), want, what="gradient forces")


def test_rational_with_overlap_gradient_and_density_in_separate_calls():
    banner("rational overlap gradient with density refused")
    import paper_1812_05264_amd as pkg
    _, H, S = overlap_cu(13, 86)
    R = rademacher(H.n, 8, config_id=86)
    fit = fit_for(H, 4, 0.3, 0.0)
    eng = engine_or_skip()
    load_overlap(eng, H, S, R)
    with pytest.raises(pkg.RfoError) as ei:
        eng.rational(0.0, fit, gradient=True, density=True)
    assert ei.value.status == "RFO_E_UNSUPPORTED"
    ok = eng.rational(0.0, fit, tol=1e-12, gradient=True)
    assert np.isfinite(ok["F"]) and np.isfinite(eng.dFdS()).all()
