"""Host-side checks of the C ABI library (no GPU needed, no compute calls)."""

import ctypes
import os
import re

import pytest

from tests.conftest import ROOT

HEADER = os.path.join(ROOT, "include", "rfo.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rfo_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for required in ("rfo_create", "rfo_destroy", "rfo_last_error", "rfo_set_hamiltonian",
                     "rfo_set_probes", "rfo_fermi_moments", "rfo_energy_and_dEdH", "rfo_hf_forces"):
        assert required in names


def test_library_exports_every_declared_symbol():
    pkg = pytest.importorskip("paper_1812_05264_amd")
    path = pkg.library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} not built: run python -m paper_1812_05264_amd.build")
    lib = ctypes.CDLL(path)
    for name in declared_symbols():
        assert hasattr(lib, name), name


def test_create_without_device_reports_error(gpu_available):
    if gpu_available:
        pytest.skip("a GPU is present")
    pkg = pytest.importorskip("paper_1812_05264_amd")
    with pytest.raises(pkg.RfoError) as ei:
        pkg.Engine()
    assert ei.value.status in ("RFO_E_DEVICE", "RFO_E_INVALID")


def test_library_exports_no_other_functions():
    """The exported functions the library defines (strong symbols) are exactly the
    ones the header declares: internal C and C++ functions are hidden.  Weak symbols
    (C++ standard-library template instantiations) and the HIP runtime's kernel
    handles (data symbols) are not functions of the library's own."""
    import shutil
    import subprocess
    pkg = pytest.importorskip("paper_1812_05264_amd")
    path = pkg.library_path()
    if not os.path.exists(path):
        pytest.fail(f"{path} not built: run python -m paper_1812_05264_amd.build")
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--defined-only", path], stdout=subprocess.PIPE, text=True,
                         check=True).stdout
    functions = set()
    for line in out.splitlines():
        parts = line.split()
        if len(parts) == 3 and parts[1] == "T":
            functions.add(parts[2])
    assert functions == set(declared_symbols()), sorted(functions ^ set(declared_symbols()))
