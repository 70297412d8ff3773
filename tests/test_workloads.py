"""Checks of the seeded input generators (CPU only)."""

import numpy as np
import pytest

from workloads import cu_cluster, rademacher, random_graph, simple_cubic
from workloads.cluster import fcc_sphere


def test_simple_cubic_structure():
    H = simple_cubic(5, disorder=1.0, config_id=3)
    assert H.n == 125 and H.nnzb == 7 * 125
    Hd = H.to_dense()
    assert np.array_equal(Hd, Hd.T)
    rows = H.block_rows()
    assert np.all(np.diff(H.col_idx.reshape(-1, 7), axis=1) > 0)
    diag = H.values[rows == H.col_idx, 0, 0]
    assert diag.size == 125 and np.max(np.abs(diag)) <= 0.5
    w = np.linalg.eigvalsh(Hd)
    assert H.e_min < w[0] and w[-1] < H.e_max
    assert simple_cubic(5, disorder=1.0, config_id=3).digest() == H.digest()
    assert simple_cubic(5, disorder=1.0, config_id=4).digest() != H.digest()


def test_simple_cubic_orderings_are_permutations():
    a = simple_cubic(6, disorder=0.7, config_id=5, ordering="natural")
    b = simple_cubic(6, disorder=0.7, config_id=5, ordering="morton")
    perm = b.meta["index_of"]
    Ad, Bd = a.to_dense(), b.to_dense()
    assert np.array_equal(Bd[np.ix_(perm, perm)], Ad)
    assert sorted(perm.tolist()) == list(range(216))


def test_fcc_sphere_selection_and_shells():
    ijk = fcc_sphere(201)
    assert ijk.shape == (201, 3)
    assert np.all(ijk.sum(axis=1) % 2 == 0)
    assert len({tuple(v) for v in ijk}) == 201
    d2 = (ijk ** 2).sum(axis=1)
    # every lattice point strictly closer than the farthest kept one is kept
    assert np.sum(d2 < d2.max()) <= 201
    cl = cu_cluster(201, config_id=5)
    cnt = np.diff(cl.row_ptr)
    assert cnt.max() == 19                     # 12 + 6 neighbours + self in the bulk
    assert cl.row_ptr[-1] == 201 + 2 * cl.pairs.shape[0]
    dist = np.sqrt(((cl.positions[cl.pairs[:, 0]] - cl.positions[cl.pairs[:, 1]]) ** 2).sum(1))
    assert np.allclose(np.unique(np.round(dist, 6)), [round(3.61 / np.sqrt(2), 6), 3.61])


def test_cu_cluster_symmetric_and_inside_interval():
    cl = cu_cluster(55, config_id=6)
    H = cl.bsr()
    Hd = H.to_dense()
    assert np.max(np.abs(Hd - Hd.T)) == 0.0
    w = np.linalg.eigvalsh(Hd)
    assert -10.0 < w[0] and w[-1] < 10.0
    assert w[-1] - w[0] > 19.0               # about 20 eV wide
    assert cu_cluster(55, config_id=6).bsr().digest() == H.digest()


def test_cu_dHdR_matches_finite_difference():
    cl = cu_cluster(19, config_id=8)
    D = cl.dH_dR()
    rows = np.repeat(np.arange(19), np.diff(cl.row_ptr))
    h = 1e-6
    for nz in [0, 5, 40, len(rows) - 1]:
        I = rows[nz]
        for d in range(3):
            p1 = cl.positions.copy()
            p1[I, d] += h
            p0 = cl.positions.copy()
            p0[I, d] -= h
            fd = (cl.values_at(p1)[nz] - cl.values_at(p0)[nz]) / (2 * h)
            assert np.max(np.abs(fd - D[nz, d])) < 1e-8


def test_rademacher_deterministic_pm1():
    R = rademacher(100, 16, config_id=2)
    assert set(np.unique(R)) == {-1.0, 1.0}
    assert np.array_equal(R, rademacher(100, 16, config_id=2))
    assert not np.array_equal(R, rademacher(100, 16, config_id=3))


def test_cu_mu_matches_its_derivation():
    import json
    import os
    from workloads.configs import CU_MU
    d = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "cu_mu.json")))
    assert CU_MU == d["mu_eV"]
    assert abs(d["electrons_per_atom_at_mu"] - 11.0) < 0.01


def test_random_graph_structure():
    H = random_graph(300, config_id=32)
    A = H.to_scipy()
    assert abs(A - A.T).max() == 0.0
    d = np.diff(H.row_ptr)
    assert d.min() == 1 and d.max() > 8          # a lone diagonal and rows past one gather chunk
    assert d[H.meta["isolated"]] == 1
    for i in range(H.n_block_rows):
        c = H.col_idx[H.row_ptr[i]:H.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    ev = np.linalg.eigvalsh(A.toarray())
    assert H.e_min < ev.min() and ev.max() < H.e_max
    assert random_graph(300, config_id=32).digest() == H.digest()
