"""Multi-color probe ensemble (Hybrid approximation, multi-color vector
ensemble; Implementation details, Welsh-Powell coloring): host construction
checked against brute force, and the estimator's exact error structure checked
with the oracle (no GPU)."""

import numpy as np

from oracle import estimator as est
from oracle import trunc
from paper_1812_05264_amd.colored import colored_probes, welsh_powell
from workloads import cu_cluster, rademacher_signs


def brute_pairs(pos, r):
    d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=2)
    return (d < r) & ~np.eye(len(pos), dtype=bool)


def test_library_coloring_on_an_irregular_cloud():
    """rfo_color_atoms on points off any lattice (many degree ties, atoms exactly at the
    radius): a proper coloring at distance < r (strict), the greedy rule in the Welsh-Powell
    order, checked against brute-force distances."""
    rng = np.random.default_rng(11)
    pos = rng.uniform(-9.0, 9.0, size=(300, 3))
    pos[1] = pos[0] + np.array([4.0, 0.0, 0.0])          # exactly at r: no edge
    r = 4.0
    c = welsh_powell(pos, r)
    adj = brute_pairs(pos, r)
    assert not adj[0, 1]
    i, j = np.nonzero(adj)
    assert np.all(c[i] != c[j])
    deg = adj.sum(axis=1)
    order = np.lexsort((np.arange(len(pos)), -deg))
    rank = np.empty(len(pos), dtype=int)
    rank[order] = np.arange(len(pos))
    for a in range(len(pos)):
        earlier = {int(c[b]) for b in np.nonzero(adj[a])[0] if rank[b] < rank[a]}
        assert c[a] == min(set(range(len(earlier) + 1)) - earlier)


def test_welsh_powell_is_a_proper_greedy_coloring():
    pos = cu_cluster(201, config_id=41).positions
    r = 6.0
    c = welsh_powell(pos, r)
    adj = brute_pairs(pos, r)
    i, j = np.nonzero(adj)
    assert np.all(c[i] != c[j])                        # no two atoms within r share a colour
    deg = adj.sum(axis=1)
    assert c.max() + 1 <= deg.max() + 1                # greedy bound
    order = np.lexsort((np.arange(len(pos)), -deg))    # decreasing degree, ties by index
    rank = np.empty(len(pos), dtype=int)
    rank[order] = np.arange(len(pos))
    for a in range(len(pos)):                          # smallest colour free of earlier neighbours
        earlier = {int(c[b]) for b in np.nonzero(adj[a])[0] if rank[b] < rank[a]}
        assert c[a] == min(set(range(len(earlier) + 1)) - earlier)
    assert np.array_equal(welsh_powell(pos, r), c)     # deterministic


def test_probe_block_structure():
    cl = cu_cluster(55, config_id=42)
    c = welsh_powell(cl.positions, 4.5)
    s = rademacher_signs(cl.n_atoms, 9, config_id=42)
    R, w = colored_probes(c, 9, s)
    q = c.max() + 1
    assert R.shape == (cl.n_atoms * 9, q * 9) and np.all(w == 1.0)
    E = R @ R.T - np.eye(R.shape[0])
    atom = np.repeat(np.arange(cl.n_atoms), 9)
    orb = np.tile(np.arange(9), cl.n_atoms)
    same = (c[atom][:, None] == c[atom][None, :]) & (orb[:, None] == orb[None, :])
    np.fill_diagonal(same, False)
    assert np.all(E[~same] == 0.0)                     # off-colour pairs cancel exactly
    assert np.all(np.abs(E[same]) == 1.0)


def test_estimate_error_is_the_same_colour_sum():
    """tr_R[X] - tr[X] = sum over same-colour, same-orbital pairs i != j of
    X_ij r_i r_j: with the truncated density P_p of the oracle the colored
    estimate of N is that exact sum (single sample, weights 1)."""
    cl = cu_cluster(43, config_id=43)
    H = cl.bsr()
    c = welsh_powell(cl.positions, 4.0)
    R, w = colored_probes(c, 9, rademacher_signs(cl.n_atoms, 9, config_id=43))
    T, mu, p = 0.4, 0.2, 60
    o = est.estimate(H, R, T, mu, p, weights=w)
    tr = trunc.observables(H.to_dense(), H.e_min, H.e_max, T, mu, p)
    P = tr["P"]
    E = R @ R.T - np.eye(R.shape[0])
    assert abs(o["N"] - (np.trace(P) + np.sum(P * E))) < 1e-10 * abs(np.trace(P))
