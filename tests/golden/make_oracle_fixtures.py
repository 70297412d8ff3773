"""Writes FP64 oracle values for the full-size Cu-like workloads (tests/golden/*.json).

At 4,000 and 16,000 atoms the oracle (scipy sparse, one core) takes minutes per
probe, too long to run beside a GPU test, so the values the full-size GPU tests
compare against are computed here once, by the oracle alone, for a few probes:

  per probe c:  N_c = sum_k alpha^f_k mu_{k,c},  E_c (alpha^{ef}),  F_c (beta^g)
                (unweighted r_c^T f(H) r_c etc. from the truncated series), and
                mu_{k,c} at sampled k.

Inputs are rebuilt from the seeded generators; each fixture stores the digest of
its Hamiltonian so that a test can check it sees the same input.

Usage: python tests/golden/make_oracle_fixtures.py [name ...]
"""

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import estimator as est  # noqa: E402
from oracle import fermi as fm  # noqa: E402
from workloads import rademacher  # noqa: E402
from workloads.configs import CONFIGS, build_hamiltonian  # noqa: E402

# (fixture name, config, number of probes drawn, probe columns kept)
FIXTURES = {
    "cu4k": ("cu4k", 128, [0, 1, 2, 3]),
    "cu16k": ("cu16k", 256, [0, 1, 2, 3]),
    "cu16k_grad16": ("cu16k_grad", 16, [0, 1]),
}
SAMPLE_K = [0, 1, 2, 3, 10, 100, 1000, 1999, 2047, 3999, 5000, 7999]


def make(name):
    cfg_name, s, cols = FIXTURES[name]
    cfg = CONFIGS[cfg_name]
    t0 = time.time()
    H, _ = build_hamiltonian(cfg)
    R = rademacher(H.n, s, config_id=cfg.config_id)[:, cols]
    p = cfg.n_terms
    mom = est.moments(est.mapped_hamiltonian(H), R, p)          # [len(cols), p]
    af, aef, bg = fm.fermi_coefficient_sets(H.e_min, H.e_max, cfg.T, cfg.mu, p)
    ks = [k for k in SAMPLE_K if k < p]
    out = {"_cite": "oracle values (estimator layer) for the workload; computed by this script",
           "config": cfg_name, "n_probes_drawn": s, "columns": cols, "n_terms": p,
           "T": cfg.T, "mu": cfg.mu, "input_digest": H.digest(),
           "N_c": (mom @ af).tolist(), "E_c": (mom @ aef).tolist(), "F_c": (mom @ bg).tolist(),
           "sample_k": ks, "moments_sampled": mom[:, ks].tolist(),
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, f"oracle_{name}.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(name, "done in", out["seconds"], "s", flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or list(FIXTURES)):
        make(nm)
