"""The C ABI from plain C: tests/c_client/rfo_client (C99, include/rfo.h only, linked
against the in-tree librfo.so by the build step) runs fermi_moments with the density
and energy_and_dEdH on seeded inputs; its outputs must match the FP64 oracle at the
parity bar, element by element, as the binding's do."""

import os
import subprocess

import numpy as np
import pytest

from oracle import estimator as est
from tests.gpu_common import TOL, banner, check_blocks, check_moments
from workloads import cu_cluster, rademacher, simple_cubic

pytestmark = pytest.mark.gpu

CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "rfo_client")


def write_input(path, H, R, T, mu, p):
    s = R.shape[1]
    with open(path, "wb") as f:
        np.array([H.n_block_rows, H.block_dim, s, p], dtype="<i8").tofile(f)
        np.array([T, mu, H.e_min, H.e_max], dtype="<f8").tofile(f)
        np.ascontiguousarray(H.row_ptr, dtype="<i8").tofile(f)
        np.ascontiguousarray(H.col_idx, dtype="<i4").tofile(f)
        np.ascontiguousarray(H.values, dtype="<f8").tofile(f)
        np.ascontiguousarray(R, dtype="<f8").tofile(f)


def read_output(path, nnzb, bd, s, p):
    d = np.fromfile(path, dtype="<f8")
    nv = nnzb * bd * bd
    assert d.size == 3 + s * p + nv + 3 + nv, d.size
    o, out = 0, {}
    out["nef"] = d[o:o + 3]; o += 3
    out["moments"] = d[o:o + s * p].reshape(s, p); o += s * p
    out["density"] = d[o:o + nv].reshape(nnzb, bd, bd); o += nv
    out["nef_grad"] = d[o:o + 3]; o += 3
    out["dFdH"] = d[o:o + nv].reshape(nnzb, bd, bd)
    return out


@pytest.mark.parametrize("case", ["sc6_ragged", "cu19"])
def test_c_client_matches_oracle(case, tmp_path):
    banner(f"C client {case}")
    if not os.path.exists(CLIENT):
        pytest.fail(f"{CLIENT} is missing: run the build step (it compiles the C client)")
    if case == "sc6_ragged":
        H, s, T, mu, p = simple_cubic(6, disorder=0.5, config_id=71), 100, 0.2, 0.1, 120
    else:
        H, s, T, mu, p = cu_cluster(19, config_id=72).bsr(), 72, 0.3, 0.2, 90
    R = rademacher(H.n, s, config_id=73)
    inp, outp = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    write_input(inp, H, R, T, mu, p)
    r = subprocess.run([CLIENT, inp, outp], stdout=subprocess.PIPE, stderr=subprocess.STDOUT,
                       text=True, timeout=120)
    assert r.returncode == 0, r.stdout
    got = read_output(outp, H.nnzb, H.block_dim, s, p)
    o = est.estimate(H, R, T, mu, p, density=True, gradient=True)
    check_moments(got["moments"], o["moments"])
    for i, key in enumerate(("N", "E", "F")):
        assert abs(got["nef"][i] - o[key]) <= TOL * max(1.0, abs(o[key])), key
        assert abs(got["nef_grad"][i] - o[key]) <= TOL * max(1.0, abs(o[key])), key
    check_blocks(got["density"], o["density"], what="density")
    check_blocks(got["dFdH"], o["dFdH"], what="dF/dH")
