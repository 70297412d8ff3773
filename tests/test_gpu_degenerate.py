"""Degenerate inputs on the GPU against the oracle: a single block row (one atom),
a pattern with no off-diagonal blocks, one probe column (the rest of the
64-wide tile is padding), series of one to a few terms, and a Hamiltonian that
is a multiple of the identity (every Chebyshev moment is T_k of one number)."""

import numpy as np
import pytest

from oracle import estimator as est
from oracle import rational as ra
from tests.gpu_common import TOL, banner, check_blocks, check_moments, engine_or_skip, load_hamiltonian, rel
from workloads import BSR, cu_cluster, rademacher

pytestmark = pytest.mark.gpu


def single_block(bd, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((bd, bd))
    A = 0.5 * (A + A.T)
    b = 1.01 * float(np.max(np.sum(np.abs(A), axis=1)))  # Gershgorin bound
    return BSR(np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32), A[None].copy(),
               bd, -b, b)


def diagonal_only(nb, bd, seed, value=None):
    rng = np.random.default_rng(seed)
    vals = np.zeros((nb, bd, bd))
    if value is None:
        d = rng.uniform(-2.0, 2.0, size=(nb, bd))
        lo, hi = -2.1, 2.1
    else:
        d = np.full((nb, bd), float(value))
        lo, hi = value - 1.0, value + 1.0
    for i in range(bd):
        vals[:, i, i] = d[:, i]
    return BSR(np.arange(nb + 1, dtype=np.int64), np.arange(nb, dtype=np.int32), vals, bd, lo, hi)


def check_all(eng, H, R, T, mu, p, weights=None):
    eng.set_probes(R, weights)
    g = eng.fermi_moments(T, mu, p, moments=True, density=True)
    o = est.estimate(H, R, T, mu, p, weights=weights, density=True, gradient=True)
    check_moments(g["moments"], o["moments"])
    for k in ("N", "E", "F"):
        assert abs(g[k] - o[k]) <= TOL * max(1.0, abs(o[k])), (k, p)
    check_blocks(g["density"], o["density"])
    for dbl in (True, False):
        eng.set_moment_doubling(dbl)
        e = eng.energy_and_dEdH(T, mu, p)
        assert abs(e["F"] - o["F"]) <= TOL * max(1.0, abs(o["F"])), (p, dbl)
        if np.any(o["dFdH"]):
            check_blocks(e["dFdH"], o["dFdH"])
        else:
            assert np.max(np.abs(e["dFdH"])) == 0.0, (p, dbl)
    eng.set_moment_doubling(True)


@pytest.mark.parametrize("bd", [1, 9])
def test_single_block_row(bd):
    banner(f"degenerate single block bd={bd}")
    H = single_block(bd, 801 + bd)
    eng = engine_or_skip()
    load_hamiltonian(eng, H)
    for s in (1, 3):
        R = rademacher(H.n, s, config_id=802)
        for p in (1, 2, 3, 8):
            check_all(eng, H, R, 0.3, 0.1, p)
    # the rational estimate on the same one-block system (S = I)
    R = rademacher(H.n, 3, config_id=803)
    eng.set_probes(R)
    import paper_1812_05264_amd as pkg
    fit = pkg.rational_fit(6, 0.3, 0.1, H.e_min, H.e_max)
    r = eng.rational(0.1, fit, tol=1e-13, density=True, gradient=True)
    o = ra.estimate(H, R, fit, density=True, gradient=True)
    for k in ("N", "E", "F"):
        assert abs(r[k] - o[k]) <= TOL * max(1.0, abs(o[k])), k
    check_blocks(r["density"], o["density"])
    check_blocks(r["dFdH"], o["dFdH"])


@pytest.mark.parametrize("bd", [1, 9])
def test_no_off_diagonal_blocks(bd):
    banner(f"degenerate diagonal-only bd={bd}")
    H = diagonal_only(300 if bd == 1 else 40, bd, 804)
    eng = engine_or_skip()
    load_hamiltonian(eng, H)
    check_all(eng, H, rademacher(H.n, 64, config_id=805), 0.2, 0.3, 40)


def test_multiple_of_identity_has_closed_form_moments():
    """H = c I: mu_{k,c} = T_k(c_hat) |r_c|^2 with c_hat the mapped value."""
    banner("degenerate constant H")
    c = 0.7
    H = diagonal_only(20, 9, 806, value=c)
    R = rademacher(H.n, 5, config_id=807)
    eng = engine_or_skip()
    load_hamiltonian(eng, H)
    p = 30
    eng.set_probes(R)
    g = eng.fermi_moments(0.1, 0.2, p, moments=True)
    ch = (2.0 * c - (H.e_min + H.e_max)) / (H.e_max - H.e_min)
    Tk = np.cos(np.arange(p) * np.arccos(ch))
    expect = np.outer(np.sum(R * R, axis=0), Tk)
    assert np.max(np.abs(g["moments"] - expect)) < 1e-12 * H.n
    check_all(eng, H, R, 0.1, 0.2, p)


def test_single_dense_probe():
    """One real (non +-1) probe column with a non-unit weight: the dense probe path
    with 63 padded columns in its tile."""
    banner("degenerate one dense probe")
    H = cu_cluster(13, config_id=808).bsr()
    rng = np.random.default_rng(809)
    R = rng.standard_normal((H.n, 1))
    eng = engine_or_skip()
    load_hamiltonian(eng, H)
    check_all(eng, H, R, 0.25, 0.0, 33, weights=np.array([0.37]))


@pytest.mark.parametrize("case", ["single_block", "diagonal_only", "one_probe"])
def test_bf16_degenerate_inputs(case):
    """BF16 MFMA steps (K chunks of one block, rows of one chunk) and the BF16
    segment gradient on degenerate inputs against the FP64 path of the same
    context: a single 9x9 block, a pattern without off-diagonal blocks, and one
    probe column (63 zero-weight padding columns in the only probe tile)."""
    banner(f"degenerate bf16 {case}")
    if case == "single_block":
        H, s = single_block(9, 810), 3
    elif case == "diagonal_only":
        H, s = diagonal_only(40, 9, 811), 64
    else:
        H, s = cu_cluster(13, config_id=812).bsr(), 1
    R = rademacher(H.n, s, config_id=813)
    eng = engine_or_skip()
    out = {}
    for prec in ("fp64", "bf16"):
        eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 9, H.e_min, H.e_max, prec)
        eng.set_probes(R)
        g = eng.fermi_moments(0.3, 0.1, 24, moments=True, density=True)
        e = eng.energy_and_dEdH(0.3, 0.1, 24)
        out[prec] = (g, e)
    (g64, e64), (g16, e16) = out["fp64"], out["bf16"]
    assert np.all(np.isfinite(g16["moments"])) and np.all(np.isfinite(e16["dFdH"]))
    assert rel(g16["moments"], g64["moments"]) < 3e-2
    assert rel(g16["density"], g64["density"]) < 3e-2
    assert abs(e16["F"] - e64["F"]) <= 1e-2 * max(1.0, abs(e64["F"]))
    if np.any(e64["dFdH"]):
        assert rel(e16["dFdH"], e64["dFdH"]) < 5e-2
