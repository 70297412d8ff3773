"""Shared helpers of the GPU tests: running the library and comparing with the oracle."""

import sys

import numpy as np
import pytest

TOL = 1e-10   # FP64 parity bar: normwise relative error on identical probes


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


def load_hamiltonian(eng, H, precision="fp64", interval=True):
    a, b = (H.e_min, H.e_max) if interval else (0.0, 0.0)
    return eng.set_hamiltonian(H.row_ptr, H.col_idx, H.values, H.block_dim, a, b, precision)
