"""Writes the FP64 oracle's free-energy gradient on the full-size 16,000-atom gradient
workload (tests/golden/oracle_cu16k_grad_G.json).

The oracle's gradient (estimator layer, Analytical free-energy derivatives: the
U-polynomial form x_j = (2 - delta_j0) sum_k beta_k U_{k-j-1}(H_hat) r with every
sum written out, no checkpoints and no reverse recurrence) is evaluated for two
probes with weight 1 each, keeping only the block rows of the 32 atoms whose
forces the finite-difference test checks (16 of lowest coordination, 16 bulk).
Stored: the gradient blocks of those rows, the forces on those atoms, F of the
two probes, and the digest of the Hamiltonian.  The forces use the symmetry of
the full gradient (G_Ja = G_aJ^T: the derivative of r^T g(H) r with respect to a
symmetric H), so one block row suffices per atom:
    force_a = -(sum_J <G_aJ, D_aJ> - sum_J <G_aJ^T, D_Ja>),  D_IJ = d H_IJ / d R_I.

Only the oracle and the seeded input generators are called.  About 25 minutes
on one core.

Usage: python tests/golden/make_oracle_grad_fixture.py
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
from workloads import finite_difference_atoms, rademacher  # noqa: E402
from workloads.configs import CONFIGS, build_hamiltonian  # noqa: E402

N_DRAWN, COLUMNS = 16, [0, 1]


def main():
    cfg = CONFIGS["cu16k_grad"]
    t0 = time.time()
    H, cl = build_hamiltonian(cfg)
    R = rademacher(H.n, N_DRAWN, config_id=cfg.config_id)[:, COLUMNS]
    p = cfg.n_terms
    low, bulk = finite_difference_atoms(H.row_ptr)
    atoms = np.concatenate([low, bulk])
    _, _, bg = fm.fermi_coefficient_sets(H.e_min, H.e_max, cfg.T, cfg.mu, p)
    w = np.ones(len(COLUMNS))
    print("inputs ready", round(time.time() - t0, 1), "s", flush=True)
    F, nz, G = est.free_energy_gradient_rows(est.mapped_hamiltonian(H), R, w, bg, p, H,
                                             H.e_min, H.e_max, atoms)
    print("gradient done", round(time.time() - t0, 1), "s", flush=True)
    rows = H.block_rows()
    cols = H.col_idx.astype(np.int64)
    D = cl.dH_dR()
    pos = {(int(r), int(c)): z for z, (r, c) in enumerate(zip(rows, cols))}
    forces = np.zeros((atoms.size, 3))
    for t, z in enumerate(nz):
        a, J = int(rows[z]), int(cols[z])
        zt = pos[(J, a)]
        dF = np.einsum("ab,dab->d", G[t], D[z]) - np.einsum("ab,dab->d", G[t].T, D[zt])
        forces[int(np.nonzero(atoms == a)[0][0])] -= dF
    out = {"_cite": "oracle gradient (estimator layer, U-polynomial form) on the block rows of "
                    "the finite-difference atoms; computed by this script",
           "config": "cu16k_grad", "n_probes_drawn": N_DRAWN, "columns": COLUMNS,
           "weights": w.tolist(), "n_terms": p, "T": cfg.T, "mu": cfg.mu,
           "input_digest": H.digest(), "e_min": H.e_min, "e_max": H.e_max,
           "atoms": atoms.tolist(), "F": F, "nz": nz.tolist(),
           "G": [float(v) for v in G.ravel()], "forces": forces.tolist(),
           "seconds": round(time.time() - t0, 1)}
    with open(os.path.join(HERE, "oracle_cu16k_grad_G.json"), "w") as f:
        json.dump(out, f)
    print("done in", out["seconds"], "s", flush=True)


if __name__ == "__main__":
    main()
