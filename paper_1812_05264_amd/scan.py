"""Chemical-potential search on stored moments.

The Chebyshev moments do not depend on T or mu, only the coefficients do
(Polynomial approximation), so once the moments of a configuration are on the
device, N(mu) at fixed T costs one coefficient and one trace kernel
(Engine.traces_at).  N is nondecreasing in mu (every f_k in the series is a
Fermi function of mu shifted by the level), so mu for a target electron count
(the paper tunes mu per cluster, Calculations) follows by bisection.  The
truncated series is monotone up to its truncation error; the search stops at
the bracket width tol.
"""


def find_mu(engine, n_target, T, lo, hi, tol=1e-9, max_iter=200):
    """mu in [lo, hi] with N(mu) = n_target, by bisection on engine.traces_at.

    The engine must hold moments from a previous fermi_moments or
    energy_and_dEdH call.  Raises ValueError when [lo, hi] does not bracket
    n_target."""
    n_lo = engine.traces_at(T, lo)["N"]
    n_hi = engine.traces_at(T, hi)["N"]
    if not (n_lo <= n_target <= n_hi):
        raise ValueError(f"N({lo}) = {n_lo}, N({hi}) = {n_hi} do not bracket {n_target}")
    for _ in range(max_iter):
        if hi - lo <= tol:
            break
        mid = 0.5 * (lo + hi)
        if engine.traces_at(T, mid)["N"] < n_target:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)
