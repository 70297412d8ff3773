"""Error conventions of the C ABI, exercised through the binding on a GPU.

Every failure here is detected on the host or by a kernel's own checks; no test
makes a kernel fault."""

import numpy as np
import pytest

from tests.gpu_common import banner, engine_or_skip, load_hamiltonian
from workloads import rademacher, simple_cubic

pytestmark = pytest.mark.gpu


def test_call_order_and_arguments():
    banner("error conventions")
    import paper_1812_05264_amd as pkg
    eng = engine_or_skip()
    with pytest.raises(pkg.RfoError) as e:
        eng.fermi_moments(0.1, 0.0, 10)
    assert e.value.status == "RFO_E_STATE"
    H = simple_cubic(4)
    with pytest.raises(pkg.RfoError) as e:
        eng.set_probes(rademacher(64, 4))
    assert e.value.status == "RFO_E_STATE"
    load_hamiltonian(eng, H)
    with pytest.raises(pkg.RfoError) as e:
        eng.fermi_moments(0.1, 0.0, 10)
    assert e.value.status == "RFO_E_STATE"
    eng.set_probes(rademacher(64, 4))
    for T, mu, p in [(0.0, 0.0, 10), (0.1, float("nan"), 10), (0.1, 0.0, 0)]:
        with pytest.raises(pkg.RfoError) as e:
            eng.fermi_moments(T, mu, p)
        assert e.value.status == "RFO_E_INVALID"
    with pytest.raises(pkg.RfoError) as e:
        eng.hf_forces(np.zeros((H.nnzb, 3, 1, 1)))
    assert e.value.status == "RFO_E_STATE"


def test_bad_patterns_are_rejected():
    banner("bad patterns")
    import paper_1812_05264_amd as pkg
    eng = engine_or_skip()
    H = simple_cubic(4)
    bad_rp = H.row_ptr.copy()
    bad_rp[5] = bad_rp[6] + 1
    col_nodiag = H.col_idx.copy()
    rows = H.block_rows()
    z = np.nonzero(rows == H.col_idx)[0][3]
    col_nodiag[z] = (col_nodiag[z] + 1) % 64
    vals_asym = H.values.copy()
    vals_asym[1, 0, 0] += 0.1
    vals_nan = H.values.copy()
    vals_nan[7, 0, 0] = np.nan
    cases = [
        (bad_rp, H.col_idx, H.values, 1, "RFO_E_INVALID"),
        (H.row_ptr, col_nodiag, H.values, 1, "RFO_E_INVALID"),
        (H.row_ptr, H.col_idx, vals_asym, 1, "RFO_E_INVALID"),
        (H.row_ptr, H.col_idx, vals_nan, 1, "RFO_E_NUMERIC"),
        (H.row_ptr, H.col_idx, H.values, 3, "RFO_E_INVALID"),
    ]
    for rp, ci, v, bd, status in cases:
        with pytest.raises(pkg.RfoError) as e:
            eng.set_hamiltonian(rp, ci, v, bd, H.e_min, H.e_max)
        assert e.value.status == status


def test_interval_too_narrow_is_numeric_error():
    banner("narrow interval")
    import paper_1812_05264_amd as pkg
    eng = engine_or_skip()
    H = simple_cubic(6, disorder=0.5, config_id=30)
    eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 1, -3.0, 3.0)
    eng.set_probes(rademacher(H.n, 8))
    with pytest.raises(pkg.RfoError) as e:
        eng.fermi_moments(0.1, 0.0, 200)
    assert e.value.status == "RFO_E_NUMERIC"


def test_gershgorin_fallback_contains_spectrum():
    banner("gershgorin")
    eng = engine_or_skip()
    H = simple_cubic(6, disorder=0.5, config_id=31)
    a, b = eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, 1, 0.0, 0.0)
    w = np.linalg.eigvalsh(H.to_dense())
    d = H.values[H.block_rows() == H.col_idx, 0, 0]
    lo, hi = d.min() - 6.0, d.max() + 6.0
    c, h = 0.5 * (lo + hi), 1.01 * 0.5 * (hi - lo)
    assert abs(a - (c - h)) < 1e-12 and abs(b - (c + h)) < 1e-12
    assert a < w[0] and w[-1] < b


def test_tuning_keys_and_values_are_validated():
    import paper_1812_05264_amd as pkg
    banner("tuning validation")
    eng = engine_or_skip()
    for key, bad in (("ppl", 3), ("grid", 4), ("sddmm_mfma", 2), ("overlap", 5), ("cplx_rows", 3)):
        with pytest.raises(pkg.RfoError):
            eng.set_tuning(key, bad)
    with pytest.raises(pkg.RfoError):
        eng._check(eng._lib.rfo_set_tuning(eng._ctx, 99, 1))
    for key in eng.TUNING:
        eng.set_tuning(key, -1)


def test_binding_refuses_buffers_of_the_wrong_size():
    """Wrong sizes and types never reach the C ABI (which would read or write past
    the buffer): the binding raises first, and the context stays usable."""
    banner("binding buffer checks")
    import torch
    eng = engine_or_skip()
    H = simple_cubic(4)
    load_hamiltonian(eng, H)
    n = H.n
    with pytest.raises(ValueError):
        eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values[:-1], 1, H.e_min, H.e_max)
    with pytest.raises(ValueError):
        eng.set_hamiltonian(H.row_ptr, H.col_idx[:-1], H.values, 1, H.e_min, H.e_max)
    with pytest.raises(ValueError):
        eng.set_probes(rademacher(n - 1, 4))
    with pytest.raises(ValueError):
        eng.set_probes(rademacher(n, 4), weights=np.ones(3))
    eng.set_probes(rademacher(n, 4))
    with pytest.raises(TypeError):
        eng.fermi_moments(0.1, 0.0, 10, density_out=torch.zeros(H.nnzb, dtype=torch.float32))
    with pytest.raises(ValueError):
        eng.fermi_moments(0.1, 0.0, 10, density_out=np.zeros(H.nnzb - 1))
    with pytest.raises(ValueError):
        eng.energy_and_dEdH(0.1, 0.0, 10, dFdH_out=np.zeros(H.nnzb + 1))
    with pytest.raises(ValueError):
        eng.hf_forces(np.zeros((H.nnzb, 2, 1, 1)))
    with pytest.raises(ValueError):
        eng.set_overlap(np.ones(H.nnzb - 1))
    g = eng.fermi_moments(0.1, 0.0, 10, density=True)
    assert np.isfinite(g["N"]) and g["density"].shape == (H.nnzb, 1, 1)
