"""Reduced-precision H.V steps (FP32 vectors, or BF16 MFMA operands with FP32
accumulation) against the FP64 oracle on the same probes.

Moments, traces, coefficients and the spectral map stay FP64 in every mode, so
the deviation comes only from the rounding of H_hat and of the vectors in the
recurrence.  The bounds below follow from that rounding: FP32 (unit roundoff
6e-8) stays many orders below them, BF16 (unit roundoff 4e-3 on every operand
of every step) is expected near 1e-3 relative on the traces over ~100 terms.
The measured errors are printed for the record.
"""

import numpy as np
import pytest

from oracle import estimator as est
from tests.gpu_common import banner, engine_or_skip, load_hamiltonian, rel
from workloads import cu_cluster, rademacher, simple_cubic

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("name,build,s,T,mu,p", [
    ("sc12", lambda: simple_cubic(12, disorder=0.8, config_id=21), 200, 0.1, 0.2, 300),
    ("cu55", lambda: cu_cluster(55, config_id=22).bsr(), 100, 0.3, 0.5, 200),
])
def test_fp32_against_oracle(name, build, s, T, mu, p):
    banner(f"fp32 {name}")
    eng = engine_or_skip()
    H = build()
    R = rademacher(H.n, s, config_id=600)
    load_hamiltonian(eng, H, precision="fp32")
    eng.set_probes(R)
    g = eng.fermi_moments(T, mu, p, density=True)
    o = est.estimate(H, R, T, mu, p, density=True)
    em, ed = rel(g["moments"], o["moments"]), rel(g["density"], o["density"])
    eN = abs(g["N"] - o["N"]) / abs(o["N"])
    print(f"fp32 {name}: moments {em:.2e} density {ed:.2e} N {eN:.2e}")
    assert em < 1e-5 and ed < 1e-5 and eN < 1e-6
    d = eng.fermi_moments(T, mu, p, moments=True)        # doubling moments
    ed2 = rel(d["moments"], o["moments"])
    eN2 = abs(d["N"] - o["N"]) / abs(o["N"])
    print(f"fp32 {name} doubling: moments {ed2:.2e} N {eN2:.2e}")
    assert ed2 < 1e-5 and eN2 < 1e-6


@pytest.mark.parametrize("name,atoms,s,p", [("cu55_s64", 55, 64, 120), ("cu201_s100", 201, 100, 120),
                                            ("cu201_s256", 201, 256, 80), ("cu13_s1000", 13, 1000, 40)])
def test_bf16_mfma_against_oracle(name, atoms, s, p):
    banner(f"bf16 {name}")
    eng = engine_or_skip()
    H = cu_cluster(atoms, config_id=23).bsr()
    R = rademacher(H.n, s, config_id=601)
    T, mu = 0.3, 0.2
    load_hamiltonian(eng, H, precision="bf16")
    eng.set_probes(R)
    g = eng.fermi_moments(T, mu, p, density=True)
    o = est.estimate(H, R, T, mu, p, density=True)
    em, ed = rel(g["moments"], o["moments"]), rel(g["density"], o["density"])
    eN = abs(g["N"] - o["N"]) / abs(o["N"])
    eE = abs(g["E"] - o["E"]) / max(1.0, abs(o["E"]))
    print(f"bf16 {name}: moments {em:.2e} density {ed:.2e} N {eN:.2e} E {eE:.2e}")
    assert np.all(g["moments"][:, 0] == o["moments"][:, 0])   # mu_0 = ||r||^2 is exact
    assert em < 3e-2 and ed < 3e-2 and eN < 1e-2 and eE < 1e-2
    d = eng.fermi_moments(T, mu, p, moments=True)        # doubling moments
    ed2 = rel(d["moments"], o["moments"])
    eN2 = abs(d["N"] - o["N"]) / abs(o["N"])
    print(f"bf16 {name} doubling: moments {ed2:.2e} N {eN2:.2e}")
    assert ed2 < 3e-2 and eN2 < 1e-2


def test_bf16_density_short_series():
    banner("bf16 density short series")
    eng = engine_or_skip()
    H = cu_cluster(55, config_id=23).bsr()
    R = rademacher(H.n, 64, config_id=603)
    load_hamiltonian(eng, H, precision="bf16")
    eng.set_probes(R)
    for p in range(1, 8):
        g = eng.fermi_moments(0.3, 0.2, p, density=True)
        o = est.estimate(H, R, 0.3, 0.2, p, density=True)
        assert rel(g["density"], o["density"]) < 3e-2, p


def test_bf16_gradient_against_fp64():
    banner("bf16 gradient")
    eng = engine_or_skip()
    cl = cu_cluster(55, config_id=26)
    H = cl.bsr()
    R = rademacher(H.n, 64, config_id=602)
    load_hamiltonian(eng, H, precision="fp64")
    eng.set_probes(R)
    g64 = eng.energy_and_dEdH(0.3, 0.4, 64)
    f64 = eng.hf_forces(cl.dH_dR())
    load_hamiltonian(eng, H, precision="bf16")
    eng.set_probes(R)
    g16 = eng.energy_and_dEdH(0.3, 0.4, 64)
    f16 = eng.hf_forces(cl.dH_dR())
    eG, eF = rel(g16["dFdH"], g64["dFdH"]), rel(f16, f64)
    print(f"bf16 gradient: dFdH {eG:.2e} forces {eF:.2e} F {abs(g16['F'] - g64['F']) / abs(g64['F']):.2e}")
    assert eG < 5e-2 and eF < 5e-2
