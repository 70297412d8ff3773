"""Nonorthogonal basis on the GPU (Polynomial approximation with S, Eq. poly_PQ;
Observable response): S^{-1} by conjugate gradients inside every step, against
the oracle's sparse-LU recurrence and generalized-eigenvalue observables."""

import numpy as np
import pytest

from oracle import overlap as ov
from tests.gpu_common import TOL, banner, check_blocks, check_moments, engine_or_skip
from workloads import BSR, cu_cluster, identity_probes, rademacher, simple_cubic
from workloads.overlap import dS_dR, overlap_values, pencil_interval

pytestmark = pytest.mark.gpu


def cu_system(n_atoms, cid):
    cl = cu_cluster(n_atoms, config_id=cid)
    H = cl.bsr()
    S = overlap_values(cl)
    a, b = pencil_interval(H, S)
    return cl, BSR(H.row_ptr, H.col_idx, H.values, 9, a, b), S


def sc_system(L, cid):
    H = simple_cubic(L, disorder=0.6, config_id=cid)
    S = np.where((H.block_rows() == H.col_idx)[:, None, None], 1.0, 0.1) * np.ones_like(H.values)
    a, b = pencil_interval(H, S)
    return BSR(H.row_ptr, H.col_idx, H.values, 1, a, b), S


def load(eng, H, S):
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, H.block_dim, H.e_min, H.e_max, "fp64")
    eng.set_overlap(S, cg_tol=1e-14)


# sc6_s340: 340 probes are three 128-column tiles (384 columns), so the CG vector kernels
# walk their column chunks (128 columns, two row lanes) more than once
@pytest.mark.parametrize("case", ["cu43", "sc6", "sc6_s340"])
def test_overlap_matches_oracle(case):
    banner(f"overlap parity {case}")
    eng = engine_or_skip()
    if case == "cu43":
        _, H, S = cu_system(43, 60)
        s, T, mu, p = 72, 0.3, 0.2, 80
    elif case == "sc6":
        H, S = sc_system(6, 61)
        s, T, mu, p = 100, 0.2, 0.1, 120
    else:
        H, S = sc_system(6, 65)
        s, T, mu, p = 340, 0.2, 0.1, 60
    R = rademacher(H.n, s, config_id=62)
    load(eng, H, S)
    eng.set_probes(R)
    g = eng.fermi_moments(T, mu, p, moments=True, density=True)
    Q = eng.density_q()
    o = ov.estimate(H, S, R, T, mu, p, density=True)
    check_moments(g["moments"], o["moments"])
    for key in ("N", "E", "F"):
        assert abs(g[key] - o[key]) <= TOL * max(1.0, abs(o[key])), key
    check_blocks(g["density"], o["density"])
    check_blocks(Q, o["density_Q"])
    it, solves = eng.cg_stats()
    print(f"{case}: {solves} CG solves, {it / max(1, solves):.1f} iterations each")
    t = eng.traces_at(0.25, 0.0)                      # stored moments, new (T, mu)
    o2 = ov.estimate(H, S, R, 0.25, 0.0, p)
    assert abs(t["N"] - o2["N"]) <= TOL * abs(o2["N"])


def test_identity_probes_give_generalized_traces():
    banner("overlap with identity probes")
    eng = engine_or_skip()
    _, H, S = cu_system(13, 63)
    T, mu, p = 0.4, 0.3, 90
    load(eng, H, S)
    eng.set_probes(identity_probes(H.n), np.ones(H.n))
    g = eng.fermi_moments(T, mu, p, density=True)
    x = ov.exact(H.to_dense(), H.with_values(S).to_dense(), T, mu, H.e_min, H.e_max, n_terms=p)
    for key in ("N", "E", "F"):
        assert abs(g[key] - x[key + "_p"]) < 1e-10 * max(1.0, abs(x[key + "_p"])), key


def test_unit_overlap_equals_orthogonal_path():
    banner("overlap S = I")
    eng = engine_or_skip()
    cl = cu_cluster(19, config_id=64)
    H = cl.bsr()
    I = np.zeros_like(H.values)
    I[H.block_rows() == H.col_idx] = np.eye(9)
    R = rademacher(H.n, 64, config_id=64)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, "fp64")
    eng.set_probes(R)
    a = eng.fermi_moments(0.3, 0.2, 70, moments=True, density=True)
    eng.set_overlap(I)
    b = eng.fermi_moments(0.3, 0.2, 70, moments=True, density=True)
    eng.set_overlap(None)
    c = eng.fermi_moments(0.3, 0.2, 70, moments=True, density=True)
    check_moments(b["moments"], a["moments"], 1e-12)
    check_blocks(b["density"], a["density"], 1e-12)
    assert np.array_equal(c["moments"], a["moments"])


def test_density_forces_match_finite_differences():
    """Identity probes and a long series: the density forces -(tr[P dH] - tr[Q dS])
    equal central differences of the exact grand potential of the pencil."""
    banner("overlap density forces vs finite differences")
    eng = engine_or_skip()
    cl, H, S = cu_system(13, 65)
    T, mu, p, h = 0.4, 0.3, 400, 1e-4
    load(eng, H, S)
    eng.set_probes(identity_probes(H.n), np.ones(H.n))
    eng.fermi_moments(T, mu, p, density=True)
    f = eng.density_forces(cl.dH_dR(), dS_dR(cl))
    f_noS = eng.density_forces(cl.dH_dR())             # without the overlap term
    assert np.max(np.abs(f - f_noS)) > 1e-3            # the tr[Q dS] term matters here

    def omega(pos):
        Hd = H.with_values(cl.values_at(pos)).to_dense()
        Sd = H.with_values(overlap_values(cl, pos)).to_dense()
        return ov.exact(Hd, Sd, T, mu, H.e_min, H.e_max)["F"]

    worst = 0.0
    for a in range(cl.n_atoms):
        for d in range(3):
            dp = np.zeros_like(cl.positions)
            dp[a, d] = h
            fd = (omega(cl.positions + dp) - omega(cl.positions - dp)) / (2 * h)
            worst = max(worst, abs(fd + f[a, d]))
    print(f"max |FD + density force| {worst:.2e} eV/A")
    assert worst < 1e-6


def test_overlap_errors():
    banner("overlap error paths")
    import paper_1812_05264_amd as pkg
    eng = engine_or_skip()
    _, H, S = cu_system(13, 66)
    with pytest.raises(pkg.RfoError):                  # no Hamiltonian yet
        eng.set_overlap(S)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, 0.0, 0.0, "fp64")
    with pytest.raises(pkg.RfoError):                  # Gershgorin interval: pass the pencil's
        eng.set_overlap(S)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, "fp32")
    with pytest.raises(pkg.RfoError):                  # FP64 only
        eng.set_overlap(S)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, "fp64")
    bad = S.copy()
    bad[0, 0, 1] += 0.5                                # S_JI != S_IJ^T
    with pytest.raises(pkg.RfoError):
        eng.set_overlap(bad)
    eng.set_overlap(S)
    eng.set_probes(rademacher(H.n, 8, config_id=66))
    with pytest.raises(pkg.RfoError):                  # no overlap gradient yet
        eng.dFdS()
    eng.energy_and_dEdH(0.3, 0.0, 20)
    D = np.zeros((H.nnzb, 3, 9, 9))
    with pytest.raises(pkg.RfoError):                  # the gradient has an overlap term
        eng.hf_forces(D)
    with pytest.raises(pkg.RfoError):                  # ... so dSdR is required
        eng.hf_forces_overlap(D, None)
    with pytest.raises(pkg.RfoError):                  # no density yet
        eng.density_forces(D)


def test_indefinite_overlap_is_an_error():
    """A symmetric but indefinite S: diagonal +-1 in equal numbers with H = 0, so every
    CG direction has p . S p = 0 exactly (alpha stays 0) and the solve cannot converge;
    the call must end with RFO_E_NUMERIC, not return numbers."""
    banner("indefinite overlap")
    import paper_1812_05264_amd as pkg
    eng = engine_or_skip()
    n = 16
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    S = np.where(np.arange(n) % 2 == 0, 1.0, -1.0).reshape(n, 1, 1)
    eng.set_hamiltonian(rp, ci, np.zeros((n, 1, 1)), 1, -1.0, 2.0, "fp64")
    eng.set_overlap(S)
    eng.set_probes(rademacher(n, 8, config_id=5))
    with pytest.raises(pkg.RfoError) as e:
        eng.fermi_moments(0.3, 0.0, 8)
    assert e.value.status == "RFO_E_NUMERIC"
    # the context stays usable: a positive definite S runs afterwards
    eng.set_overlap(np.abs(S))
    g = eng.fermi_moments(0.3, 0.0, 8)
    assert np.isfinite(g["N"])


@pytest.mark.parametrize("case", ["cu43_s72", "cu19_dense", "sc6_s100", "cu13_p2"])
def test_overlap_gradient_matches_oracle(case):
    """dF~/dH and dF~/dS with an overlap (Analytical free-energy derivatives, Eq.
    polynomial_response) against the oracle's form of the same derivative (left vectors
    T_j(S^{-1} H_hat) r, right vectors S^{-1} times U-polynomial sums), both as symmetric parts;
    several checkpoint segments (cu43: 79 gradient terms in segments of 9), dense probes with
    unequal weights, 1x1 blocks, and the shortest series with a gradient term."""
    banner(f"overlap gradient parity {case}")
    eng = engine_or_skip()
    w = None
    if case == "cu43_s72":
        _, H, S = cu_system(43, 67)
        R = rademacher(H.n, 72, config_id=68)
        T, mu, p = 0.3, 0.2, 80
    elif case == "cu19_dense":
        _, H, S = cu_system(19, 69)
        R = rademacher(H.n, 37, config_id=70) * (1.0 + 0.25 * np.cos(np.arange(H.n)))[:, None]
        w = np.linspace(0.5, 1.5, 37) / 37
        T, mu, p = 0.3, 0.2, 31
    elif case == "sc6_s100":
        H, S = sc_system(6, 71)
        R = rademacher(H.n, 100, config_id=72)
        T, mu, p = 0.2, 0.1, 60
    else:
        _, H, S = cu_system(13, 73)
        R = rademacher(H.n, 16, config_id=74)
        T, mu, p = 0.3, 0.2, 2
    load(eng, H, S)
    eng.set_probes(R, w)
    g = eng.energy_and_dEdH(T, mu, p)
    GS = eng.dFdS()
    F, oH, oS = ov.free_energy_gradient(H, S, R, T, mu, p, weights=w)
    assert abs(g["F"] - F) <= TOL * max(1.0, abs(F))
    eH = check_blocks(g["dFdH"], oH, what="dF/dH")
    eS = check_blocks(GS, oS, what="dF/dS")
    print(f"{case}: dF/dH {eH:.2e}, dF/dS {eS:.2e} per block")
    again = eng.energy_and_dEdH(T, mu, p)
    assert np.array_equal(again["dFdH"], g["dFdH"]) and np.array_equal(eng.dFdS(), GS)


def test_overlap_gradient_forces_match_finite_differences():
    """Forces -(sum <dF~/dH, dH/dR> + sum <dF~/dS, dS/dR>) from the GPU gradient against central
    differences of the oracle's F~ in the atom positions (same probes, fixed interval)."""
    banner("overlap gradient forces vs finite differences")
    eng = engine_or_skip()
    cl, H, S = cu_system(13, 75)
    R = rademacher(H.n, 16, config_id=76)
    T, mu, p, h = 0.4, 0.3, 60, 1e-4
    load(eng, H, S)
    eng.set_probes(R)
    eng.energy_and_dEdH(T, mu, p)
    f = eng.hf_forces_overlap(cl.dH_dR(), dS_dR(cl))

    def F_at(pos):
        return ov.estimate(H.with_values(cl.values_at(pos)), overlap_values(cl, pos), R, T, mu, p)["F"]

    worst = 0.0
    for a in range(cl.n_atoms):
        for d in range(3):
            dp = np.zeros_like(cl.positions)
            dp[a, d] = h
            fd = (F_at(cl.positions + dp) - F_at(cl.positions - dp)) / (2 * h)
            worst = max(worst, abs(fd + f[a, d]))
    print(f"max |FD + gradient force| {worst:.2e} eV/A (largest force {np.max(np.abs(f)):.2e})")
    assert worst < 1e-6
