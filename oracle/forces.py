"""Hellmann-Feynman forces from the free-energy gradient (Observable response, S = I).

dF/dlambda = tr[P dH/dlambda], with P replaced by the estimator's gradient
G = dF/dH on the block pattern.  For a two-centre model H_IJ = h(R_I - R_J),
d H_IJ / d R_a = (delta_aI - delta_aJ) D_IJ with D_IJ = d H_IJ / d R_I, so
    dF/dR_a = sum_J <G_aJ, D_aJ> - sum_I <G_Ia, D_Ia>,   force_a = -dF/dR_a,
where <A, B> = sum_{ij} A_ij B_ij over the block.

Test infrastructure only (see the package docstring).
"""

import numpy as np


def hf_forces(bsr, G, dHdR):
    """G [nnzb, bd, bd], dHdR [nnzb, 3, bd, bd] -> forces [n_block_rows, 3]."""
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    contrib = np.einsum("zab,zdab->zd", np.asarray(G), np.asarray(dHdR))   # <G_IJ, D_IJ> per direction
    dF = np.zeros((bsr.n_block_rows, 3))
    np.add.at(dF, rows, contrib)
    np.add.at(dF, cols, -contrib)
    return -dF
