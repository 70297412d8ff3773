"""Compiles tests/c_client/rfo_client.c (a plain C99 client of include/rfo.h) against the
in-tree librfo.so.  Called by the repository's build step; the binary is not committed."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
PKG = os.path.join(ROOT, "paper_1812_05264_amd")
SRC = os.path.join(HERE, "rfo_client.c")
BIN = os.path.join(HERE, "rfo_client")


def build_client() -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-pedantic",
           "-I", os.path.join(ROOT, "include"), SRC, "-o", BIN + ".tmp",
           "-L", PKG, "-lrfo", "-Wl,-rpath,$ORIGIN/../../paper_1812_05264_amd",
           "-Wl,-rpath-link,/opt/rocm/lib"]
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("C client build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build_client())
