"""Randomized Chebyshev Fermi-operator expansion on MI355X (gfx950).

The compute path is the HIP library librfo.so (include/rfo.h); this package holds
its ctypes binding and a torch.autograd.Function around the free-energy gradient.

Typical use, with H in block-sparse rows and a probe block R [n][s]:

    eng = Engine(0)
    eng.set_hamiltonian(row_ptr, col_idx, values, block_dim, e_min, e_max, "fp64")
    eng.set_probes(R)                         # +-1 probes are kept as sign bits
    out = eng.fermi_moments(T, mu, n_terms, moments=True, density=True)
    # out["N"], out["E"], out["F"], out["moments"] [s][p], out["density"] [nnzb][bd][bd]
    g = eng.energy_and_dEdH(T, mu, n_terms)   # g["F"], g["dFdH"]
    forces = eng.hf_forces(dH_dR)             # [n_block_rows][3]
"""

from ._rfo import Engine, RfoError, library_path, load, PRECISIONS, rational_fit  # noqa: F401
from .scan import find_mu  # noqa: F401
from .colored import colored_probes, welsh_powell  # noqa: F401

__all__ = ["Engine", "RfoError", "library_path", "load", "PRECISIONS", "find_mu",
           "colored_probes", "welsh_powell", "rational_fit"]
