"""The plain C client of the C ABI builds from include/rfo.h alone (C99, -pedantic,
warnings as errors) and reports bad input with its own exit status; its results are
checked on the GPU (test_gpu_c_client.py)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "c_client"))


def test_client_builds_and_rejects_a_short_input(tmp_path):
    from build_client import build_client
    exe = build_client()
    bad = tmp_path / "in.bin"
    bad.write_bytes(b"\x01\x02")
    r = subprocess.run([exe, str(bad), str(tmp_path / "out.bin")], stdout=subprocess.PIPE,
                       stderr=subprocess.STDOUT, text=True, timeout=60)
    assert r.returncode == 2 and "short header" in r.stdout
    r = subprocess.run([exe], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       timeout=60)
    assert r.returncode == 2 and "usage" in r.stdout
