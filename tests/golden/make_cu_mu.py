"""Derives the chemical potential of the Cu-like workloads with the FP64 oracle.

mu is chosen so that the 4,000-atom Cu-like cluster holds 11 electrons per atom
(spin included) at kT = 0.05 eV: the stochastic moments mu_{k,c} = r_c^T T_k(H_hat) r_c
do not depend on mu, so they are computed once (8 Rademacher probes from a
dedicated stream, 1500 Chebyshev terms) and N(mu) = sum_c w_c sum_k alpha^f_k(mu) mu_{k,c}
is bisected.  The result is rounded to 1e-3 eV and written to cu_mu.json; the
workload definitions carry the same number.

Usage: python tests/golden/make_cu_mu.py
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
from workloads import cu_cluster, rademacher  # noqa: E402

N_ATOMS, T, P, S, TARGET = 4000, 0.05, 1500, 8, 11.0


def main():
    t0 = time.time()
    H = cu_cluster(N_ATOMS, config_id=2).bsr()
    R = rademacher(H.n, S, config_id=2, stream=7)
    mom = est.moments(est.mapped_hamiltonian(H), R, P)
    w = est.default_weights(S)
    m = w @ mom

    def electrons(mu):
        af = fm.chebyshev_coefficients(lambda e: fm.fermi(e, T, mu), H.e_min, H.e_max, P)
        return float(af @ m)

    lo, hi = H.e_min, H.e_max
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if electrons(mid) < TARGET * N_ATOMS:
            lo = mid
        else:
            hi = mid
    mu = round(0.5 * (lo + hi), 3)
    out = {"_cite": "workload choice: Cu-like filling of 11 electrons per atom (3d10 4s1), spin "
                    "factor 2 as in the Fermi function of the paper's Methods",
           "mu_eV": mu, "electrons_per_atom_at_mu": electrons(mu) / N_ATOMS,
           "n_atoms": N_ATOMS, "kT_eV": T, "n_terms": P, "probes": S,
           "input_digest": H.digest(), "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "cu_mu.json"), "w") as f:
        json.dump(out, f, indent=2)
    print(json.dumps(out, indent=2))


if __name__ == "__main__":
    main()
