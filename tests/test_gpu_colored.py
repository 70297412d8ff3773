"""Multi-color probe ensemble on the GPU (Hybrid approximation, multi-color
vector ensemble): the structured +-1/0 probes go through the same probe input,
so moments, density, gradient and forces must match the oracle on the same
probes, and the estimate's error must be exactly the same-colour sum of the
truncated density matrix."""

import numpy as np
import pytest

from oracle import estimator as est
from oracle import forces as ofo
from oracle import trunc
from tests.gpu_common import TOL, banner, check_blocks, check_moments, check_rows, engine_or_skip, load_hamiltonian
from workloads import cu_cluster, rademacher_signs

pytestmark = pytest.mark.gpu


def colored(cl, r_max, config_id):
    from paper_1812_05264_amd.colored import colored_probes, welsh_powell
    c = welsh_powell(cl.positions, r_max)
    return colored_probes(c, 9, rademacher_signs(cl.n_atoms, 9, config_id=config_id))


@pytest.mark.parametrize("r_max", [4.5, 5.5])
@pytest.mark.parametrize("doubling", [True, False])
def test_colored_probes_match_oracle(doubling, r_max):
    """r_max 4.5: 8 colours, 72 columns; 5.5: 16 colours, 144 columns, whose gradient runs
    the last 16 columns as a probe batch of their own."""
    banner(f"multi-color probes vs oracle doubling={doubling} r_max={r_max}")
    eng = engine_or_skip()
    eng.set_moment_doubling(doubling)
    cl = cu_cluster(55, config_id=44)
    H = cl.bsr()
    R, w = colored(cl, r_max, 44)
    load_hamiltonian(eng, H)
    eng.set_probes(R, w)
    T, mu, p = 0.3, 0.3, 90
    g = eng.fermi_moments(T, mu, p, moments=True, density=True)
    o = est.estimate(H, R, T, mu, p, weights=w, density=True, gradient=True)
    check_moments(g["moments"], o["moments"])
    check_blocks(g["density"], o["density"])
    for key in ("N", "E", "F"):
        assert abs(g[key] - o[key]) <= TOL * max(1.0, abs(o[key])), key
    e = eng.energy_and_dEdH(T, mu, p)
    check_blocks(e["dFdH"], o["dFdH"])
    D = cl.dH_dR()
    check_rows(eng.hf_forces(D), ofo.hf_forces(H, o["dFdH"], D), what="forces")


def test_colored_error_is_the_same_colour_sum():
    banner("multi-color error structure vs coloring radius")
    eng = engine_or_skip()
    cl = cu_cluster(201, config_id=45)
    H = cl.bsr()
    load_hamiltonian(eng, H)
    T, mu, p = 0.3, 0.3, 120
    P = trunc.observables(H.to_dense(), H.e_min, H.e_max, T, mu, p)["P"]
    errs = []
    for r_max in (3.0, 6.0, 9.0):
        R, w = colored(cl, r_max, 45)
        eng.set_probes(R, w)
        g = eng.fermi_moments(T, mu, p)
        E = R @ R.T - np.eye(R.shape[0])
        err = g["N"] - np.trace(P)
        assert abs(err - np.sum(P * E)) < 1e-9 * np.trace(P), r_max
        errs.append((r_max, R.shape[1], err))
    print("coloring radius, probe columns, N error:", errs)


@pytest.mark.parametrize("prec", ["fp64", "bf16"])
def test_library_built_colored_probes_equal_the_host_block(prec):
    """rfo_set_colored_probes builds on the device the block colored_probes builds on the
    host: the same moments, traces and gradient bit for bit."""
    banner(f"library-built colored probes {prec}")
    from paper_1812_05264_amd.colored import colored_probes, welsh_powell
    eng = engine_or_skip()
    cl = cu_cluster(201, config_id=46)
    H = cl.bsr()
    c = welsh_powell(cl.positions, 6.0)
    signs = rademacher_signs(cl.n_atoms, 9, config_id=46)
    R, w = colored_probes(c, 9, signs)
    load_hamiltonian(eng, H, precision=prec)
    T, mu, p = 0.3, 0.3, 80
    eng.set_probes(R, w)
    a = eng.fermi_moments(T, mu, p, moments=True)
    ga = eng.energy_and_dEdH(T, mu, p)
    eng.set_colored_probes(c, 9, signs)
    b = eng.fermi_moments(T, mu, p, moments=True)
    gb = eng.energy_and_dEdH(T, mu, p)
    assert np.array_equal(a["moments"], b["moments"])
    assert a["F"] == b["F"] and ga["F"] == gb["F"]
    assert np.array_equal(ga["dFdH"], gb["dFdH"])
