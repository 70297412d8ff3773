"""Host logic of the mu search (no GPU): bisection on a monotone N(mu)."""

import math

import pytest

from paper_1812_05264_amd.scan import find_mu


class FakeEngine:
    """N(mu) of 100 two-fold levels at T: the Fermi sum itself."""

    def __init__(self):
        self.levels = [-2.0 + 4.0 * i / 99 for i in range(100)]
        self.calls = 0

    def traces_at(self, T, mu):
        self.calls += 1
        n = sum(2.0 / (1.0 + math.exp((e - mu) / T)) for e in self.levels)
        return {"N": n, "E": 0.0, "F": 0.0}


def test_find_mu_hits_target_count():
    eng = FakeEngine()
    mu = find_mu(eng, 120.0, 0.1, -3.0, 3.0, tol=1e-12)
    assert abs(eng.traces_at(0.1, mu)["N"] - 120.0) < 1e-9
    assert eng.calls < 60


def test_find_mu_rejects_bad_bracket():
    with pytest.raises(ValueError):
        find_mu(FakeEngine(), 500.0, 0.1, -3.0, 3.0)
