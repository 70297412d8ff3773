"""Padding probe columns of dense probe blocks.

Probe blocks are padded to a multiple of the kernels' probe tiles with weight-zero columns.
For dense probes those columns are zero, so every vector of the recurrence is zero there and
the step kernels skip their loads; the outer products skip every weight-zero column.  Sign-bit
probes (entries exactly +-1) carry -1 in their padding columns and are computed in full.

The check needs no tolerance: a dense block equal to R / 2 for Rademacher R takes the skipping
path, R itself the full one, and scaling by a power of two is exact in every precision, so the
moments, density blocks, traces and gradient of R / 2 are exactly a quarter of those of R.
"""

import numpy as np
import pytest

from tests.gpu_common import banner, engine_or_skip, load_hamiltonian
from workloads import cu_cluster, rademacher, simple_cubic

pytestmark = pytest.mark.gpu

CASES = [
    ("sc6_fp64", lambda: simple_cubic(6, disorder=0.6, config_id=41), "fp64", 100),
    ("sc6_fp32", lambda: simple_cubic(6, disorder=0.6, config_id=41), "fp32", 37),
    ("cu55_fp64", lambda: cu_cluster(55, config_id=42).bsr(), "fp64", 100),
    ("cu55_fp64_s200", lambda: cu_cluster(55, config_id=42).bsr(), "fp64", 200),
    ("cu55_fp32", lambda: cu_cluster(55, config_id=42).bsr(), "fp32", 70),
    ("cu55_bf16", lambda: cu_cluster(55, config_id=42).bsr(), "bf16", 100),
    ("cu55_bf16x2", lambda: cu_cluster(55, config_id=42).bsr(), "bf16x2", 20),
]


def run(H, prec, R, T, mu, p, doubling, adjoint_bytes=None):
    eng = engine_or_skip()
    load_hamiltonian(eng, H, precision=prec)
    eng.set_probes(R)
    eng.set_moment_doubling(doubling)
    m = eng.fermi_moments(T, mu, p, moments=True, density=True)
    if adjoint_bytes is not None:
        eng.set_tuning("adjoint_bytes", adjoint_bytes)
    g = eng.energy_and_dEdH(T, mu, p)
    eng.close()
    return m, g


@pytest.mark.parametrize("name,build,prec,s", CASES)
def test_dense_half_probes_are_exactly_a_quarter(name, build, prec, s):
    banner(f"padding {name} s={s}")
    H = build()
    R = rademacher(H.n, s, config_id=43)
    T, mu, p = 0.3, 0.2, 70
    for doubling in (True, False):
        ma, ga = run(H, prec, R, T, mu, p, doubling)
        mb, gb = run(H, prec, 0.5 * R, T, mu, p, doubling)
        assert np.array_equal(mb["moments"], 0.25 * ma["moments"]), doubling
        assert np.array_equal(mb["density"], 0.25 * ma["density"]), doubling
        for k in ("N", "E", "F"):
            assert mb[k] == 0.25 * ma[k], (k, doubling)
            assert gb[k] == 0.25 * ga[k], (k, doubling)
        assert np.array_equal(gb["dFdH"], 0.25 * ga["dFdH"]), doubling


def test_dense_half_probes_in_batches():
    """The adjoint's probe batches: 200 columns in batches of 64 (the last one 8 columns,
    padded to 64), for sign-bit and dense probes alike."""
    banner("padding with probe batches")
    import re
    import paper_1812_05264_amd as pkg
    H = cu_cluster(55, config_id=44).bsr()
    R = rademacher(H.n, 200, config_id=45)
    T, mu, p = 0.3, 0.2, 40
    eng = engine_or_skip()
    load_hamiltonian(eng, H)
    eng.set_probes(R)
    eng.set_tuning("adjoint_bytes", 1)
    with pytest.raises(pkg.RfoError) as err:
        eng.energy_and_dEdH(T, mu, p)
    eng.close()
    per64 = int(re.search(r"needs (\d+) bytes of vectors for one batch of 64", str(err.value)).group(1))
    _, ga = run(H, "fp64", R, T, mu, p, True, adjoint_bytes=per64 * 3 // 2)
    _, gb = run(H, "fp64", 0.5 * R, T, mu, p, True, adjoint_bytes=per64 * 3 // 2)
    assert gb["F"] == 0.25 * ga["F"]
    assert np.array_equal(gb["dFdH"], 0.25 * ga["dFdH"])
