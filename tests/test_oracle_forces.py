"""Pins of the oracle's Hellmann-Feynman force contraction (CPU only)."""

import numpy as np
import pytest

from oracle import estimator as est
from oracle import forces
from workloads import cu_cluster, rademacher


@pytest.fixture(scope="module")
def cl43():
    return cu_cluster(43, config_id=12)


def _F(cl, pos, R, T, mu, p):
    return est.estimate(cl.bsr(pos), R, T, mu, p)["F"]


def test_forces_sum_to_zero_and_match_finite_differences(cl43):
    cl = cl43
    H = cl.bsr()
    R = rademacher(H.n, 3, config_id=82)
    T, mu, p = 0.4, 0.1, 80
    G = est.estimate(H, R, T, mu, p, gradient=True)["dFdH"]
    Fa = forces.hf_forces(H, G, cl.dH_dR())
    assert np.max(np.abs(Fa.sum(axis=0))) < 1e-12 * np.max(np.abs(Fa))
    rng = np.random.default_rng(3)
    d = rng.standard_normal(cl.positions.shape)
    h = 1e-4
    fd = (_F(cl, cl.positions + h * d, R, T, mu, p) - _F(cl, cl.positions - h * d, R, T, mu, p)) / (2 * h)
    assert abs(fd + np.sum(Fa * d)) < 1e-6 * max(1.0, np.abs(Fa).sum())
    # single-atom displacement
    for atom in (0, 21):
        e = np.zeros_like(cl.positions)
        e[atom, 1] = 1.0
        fd = (_F(cl, cl.positions + h * e, R, T, mu, p) - _F(cl, cl.positions - h * e, R, T, mu, p)) / (2 * h)
        assert abs(fd + Fa[atom, 1]) < 1e-6


def test_forces_agree_with_autograd_of_the_model(cl43):
    torch = pytest.importorskip("torch")
    cl = cl43
    H = cl.bsr()
    R = rademacher(H.n, 2, config_id=83)
    G = est.estimate(H, R, 0.4, 0.1, 40, gradient=True)["dFdH"]
    pos = torch.tensor(cl.positions, dtype=torch.float64, requires_grad=True)
    vals = cl.values_torch(pos)
    assert np.max(np.abs(vals.detach().numpy() - H.values)) < 1e-14
    (vals * torch.as_tensor(G)).sum().backward()
    Fa = forces.hf_forces(H, G, cl.dH_dR())
    assert np.max(np.abs(pos.grad.numpy() + Fa)) < 1e-12 * max(1.0, np.abs(Fa).max())
