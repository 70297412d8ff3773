"""Shared helpers of the GPU tests: running the library and comparing with the oracle.

Parity is checked two ways, both at the FP64 bar TOL:
  * normwise: ||got - want||_F / ||want||_F over the whole array (rel);
  * element by element (check_* helpers), so that a wrong late moment, a wrong small block
    or a wrong tail probe cannot hide behind the norm of the large entries:
      moments [s, p]      |got - want| <= tol * max(|want|, sqrt(mu_0)) per moment, where
                          sqrt(mu_0) = ||r_c|| is the size of a random-probe moment r^T T_k r
                          (its rounding error is of order u ||r_c|| ||y_k||, ||y_k|| <= ||r_c||);
      blocks [nnzb, a, b] max_ab |got - want| <= tol * max_ab |want| per block;
      rows [m, d]         the same per row (forces per atom, per-probe traces).
"""

import sys

import numpy as np
import pytest

TOL = 1e-10   # FP64 parity bar on identical probes


def engine_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1812_05264_amd as pkg
    return pkg.Engine(0)


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


def group_err(got, want):
    """Worst over the leading axis of max|got_g - want_g| / max|want_g| (a group whose wanted
    values are all zero must be matched exactly)."""
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    assert got.shape == want.shape, (got.shape, want.shape)
    if got.size == 0:
        return 0.0
    g = got.reshape(got.shape[0], -1)
    w = want.reshape(want.shape[0], -1)
    d = np.max(np.abs(g - w), axis=1)
    sc = np.max(np.abs(w), axis=1)
    if np.any((sc == 0) & (d != 0)):
        return float("inf")
    r = np.divide(d, sc, out=np.zeros_like(d), where=sc > 0)
    return float(np.max(r))


def moment_err(got, want):
    """Moments [s, p] (or one probe's [p]), mu_0 = ||r_c||^2 first."""
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    want = np.atleast_2d(np.asarray(want, dtype=np.float64))
    assert got.shape == want.shape, (got.shape, want.shape)
    floor = np.sqrt(np.abs(want[:, :1]))
    sc = np.maximum(np.abs(want), floor)
    return float(np.max(np.abs(got - want) / np.where(sc > 0, sc, 1.0)))


def check_moments(got, want, tol=TOL, what="moments"):
    e_norm, e_el = rel(got, want), moment_err(got, want)
    assert e_norm < tol and e_el < tol, f"{what}: normwise {e_norm:.2e}, per moment {e_el:.2e}"
    return e_el


def check_blocks(got, want, tol=TOL, what="blocks"):
    e_norm, e_el = rel(got, want), group_err(got, want)
    assert e_norm < tol and e_el < tol, f"{what}: normwise {e_norm:.2e}, per block {e_el:.2e}"
    return e_el


check_rows = check_blocks


def load_hamiltonian(eng, H, precision="fp64", interval=True):
    a, b = (H.e_min, H.e_max) if interval else (0.0, 0.0)
    return eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, H.block_dim, a, b, precision)
