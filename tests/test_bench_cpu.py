"""Host-side pieces of bench.py: the algorithmic byte count and the kernel digest that
ties the committed counter traffic to the step kernel's code."""

import os

import numpy as np

import bench
from workloads import simple_cubic


def test_accumulator_updates_and_step_bytes():
    # three terms per update and one at the last step: p = 2048 gives 683 updates in 2047 steps
    assert bench.acc_updates(2048) == 683
    assert bench.acc_updates(4) == 1 and bench.acc_updates(5) == 2
    H = simple_cubic(4)
    s, p = 64, 2048
    vec = H.n * s * 8
    h = H.nnzb * 8 + H.nnzb * 4 + (H.n_block_rows + 1) * 8
    bits = H.n * s / 8.0
    assert bench.step_bytes(H, s, 8, 8, density=False) == h + 3 * vec + bits
    assert np.isclose(bench.step_bytes(H, s, 8, 8, density=True, p=p), h + (3 + 2 * 683 / 2047) * vec + bits)


def test_kernel_digest_follows_code_not_comments():
    csrc = os.path.join(bench.ROOT, "paper_1812_05264_amd", "csrc")
    files = {f: open(os.path.join(csrc, f), "rb").read() for f in ("k_step.hip", "device_util.h", "rfo_internal.h")}
    base = bench.kernel_digest(lambda f: files[f])
    assert base == bench.kernel_digest()
    commented = dict(files)
    commented["k_step.hip"] = files["k_step.hip"].replace(b"namespace rfo {", b"namespace rfo {  // note\n/* more */", 1)
    assert bench.kernel_digest(lambda f: commented[f]) == base
    changed = dict(files)
    changed["k_step.hip"] = files["k_step.hip"].replace(b"namespace rfo {", b"namespace rfo { int unused_;", 1)
    assert bench.kernel_digest(lambda f: changed[f]) != base
    # only the StepArgs struct of the internal header counts
    other = dict(files)
    other["rfo_internal.h"] = files["rfo_internal.h"] + b"\nint another_declaration();\n"
    assert bench.kernel_digest(lambda f: other[f]) == base
