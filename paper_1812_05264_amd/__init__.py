"""Randomized Chebyshev Fermi-operator expansion on MI355X (gfx950).

The compute path is the HIP library librfo.so (include/rfo.h); this package holds
its ctypes binding and a torch.autograd.Function around the free-energy gradient.
"""

from ._rfo import Engine, RfoError, library_path, load, PRECISIONS, rational_fit  # noqa: F401
from .scan import find_mu  # noqa: F401
from .colored import colored_probes, welsh_powell  # noqa: F401

__all__ = ["Engine", "RfoError", "library_path", "load", "PRECISIONS", "find_mu",
           "colored_probes", "welsh_powell", "rational_fit"]
