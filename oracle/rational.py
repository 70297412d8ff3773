"""Rational (pole) expansion of the Fermi-Dirac and free-energy functions.

Follows the paper's Rational approximation subsection and the rational part of
Analytical free-energy derivatives:

  * residue-pole form (Eq. rational_fit), here with the constant / linear part
    that an approximation on a finite interval carries:
        f(x) ~ f0 + 2 Re sum_k w_k / (x - z_k),
        g(x) ~ g0 + g1 x + 2 Re sum_k tau_k / (x - z_k),
    both on the same poles z_k (Im z_k > 0);
  * the linear systems of Eq. rational_PQ with S = I:  (H - z_k) g_k = y,
        P y = f0 y + 2 Re sum_k w_k g_k,
        Q y = f0 H y + 2 Re [ y sum_k w_k + sum_k w_k z_k g_k ],
    solved here exactly by a sparse LU factorization (library primitive);
  * with an overlap S (Eq. rational_PQ as printed): (H - z_k S) g_k = y,
        P y = f0 S^{-1} y + 2 Re sum_k w_k g_k,   Q y = S^{-1} H P y,
    N = tr[P S], E = tr[P H], F = tr g(H S^{-1}) estimated on the probes as
    (S r).(P r), (H r).(P r) and g0 r.r + g1 (H r).(S^{-1} r) + 2 Re sum_k tau_k (S r).g_k;
  * the rational free-energy primitive F(y) = g0 y.y + g1 y.H y
        + 2 Re sum_k tau_k y^T G(z_k) y and its derivative (Eq.
    rational_derivative with dS = 0): dF(y)/dH_ab = g1 y_a y_b
        - 2 Re sum_k tau_k g_{k,a} g_{k,b}   (G(z)^T = G(z) for symmetric H);
    with an overlap, the derivative with respect to H and S (gradient_overlap).

The paper's fastest fit is a numerical one whose poles are not printed.  The
fit here is the analytical kind the paper also names, valid on a finite
spectral interval [e_min, e_max] and applicable to both f and g: a
contour-integral (trapezoid) rule on a conformal map of an annulus
(Hale, Higham and Trefethen, SIAM J. Numer. Anal. 46 (2008), their first
method for functions analytic off (-inf, 0]), applied to the even parts of
f and g written as functions of u = (x - mu)^2:
    f(x) = 1 - X h(X^2),        h(u) = tanh(sqrt(u)/(2T)) / sqrt(u),
    g(x) = X - 2T ln 2 - 2T l(X^2),  l(u) = ln cosh(sqrt(u)/(2T)),      X = x - mu.
h and l are analytic in u off (-inf, -(pi T)^2], so with xi = u + (pi T)^2 the
rule of that paper applies on [m, M] = [(pi T)^2, D^2 + (pi T)^2],
D = max(|e_min - mu|, |e_max - mu|).  Each of the n_nodes quadrature nodes xi_j
(upper half plane) gives the two poles mu + s_j and mu - conj(s_j),
s_j = sqrt(xi_j - m), so the fit has 2 n_nodes pole pairs.

Test infrastructure only (see the package docstring).
"""

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import scipy.special as ss

from . import estimator as est


def jacobi_sncndn(x, y, m):
    """sn, cn, dn of the complex argument x + i y (x, y real arrays), parameter m = k^2.

    Jacobi's imaginary transformation gives the functions at i y from those at y
    with the complementary parameter 1 - m; the addition theorems combine them
    with the values at x (library routine for real arguments)."""
    s, c, d, _ = ss.ellipj(np.asarray(x, dtype=np.float64), m)
    s1, c1, d1, _ = ss.ellipj(np.asarray(y, dtype=np.float64), 1.0 - m)
    sb, cb, db = 1j * s1 / c1, 1.0 / c1, d1 / c1
    den = 1.0 - m * s * s * sb * sb
    sn = (s * cb * db + sb * c * d) / den
    cn = (c * cb - s * d * sb * db) / den
    dn = (d * db - m * s * c * sb * cb) / den
    return sn, cn, dn


def contour_fit(n_nodes, T, mu, e_min, e_max):
    """Poles and residues of the rational approximations of f and g on [e_min, e_max].

    Returns dict(poles [2n], res_f [2n], res_g [2n], f0, g0, g1); all poles have
    Im > 0 and the approximants are f0 + 2 Re sum res_f/(x - z) and
    g0 + g1 x + 2 Re sum res_g/(x - z)."""
    if n_nodes < 1:
        raise ValueError("need at least one node")
    D = max(abs(e_min - mu), abs(e_max - mu))
    m = (np.pi * T) ** 2
    M = D * D + m
    q = np.sqrt(M / m)
    k = (q - 1.0) / (q + 1.0)
    kp2 = 4.0 * q / (q + 1.0) ** 2          # 1 - k^2, formed without cancellation
    K = ss.ellipkm1(kp2)                    # K(k^2)
    Kp = ss.ellipk(kp2)                     # K(1 - k^2)
    # midpoints of n_nodes equal steps along Im t = K'/2, Re t in [-K, K]
    t = -K + (np.arange(n_nodes) + 0.5) * (2.0 * K / n_nodes)
    sn, cn, dn = jacobi_sncndn(t, np.full(n_nodes, 0.5 * Kp), k * k)
    c = np.sqrt(m * M)
    xi = c * (1.0 / k + sn) / (1.0 / k - sn)        # nodes in the upper half plane
    dxi = cn * dn / (1.0 / k - sn) ** 2              # d xi / dt without the factor 2c/k
    # F(A) ~ -(1/pi) Im sum_j (2K/n) F(xi_j) (xi_j - A)^{-1} (2c/k) dxi_j
    C = 4.0 * K * c / (np.pi * n_nodes * k)
    s = np.sqrt(xi - m)                              # first quadrant
    w = s / (2.0 * T)
    e2 = np.exp(-2.0 * w)
    h = (1.0 - e2) / (1.0 + e2) / s                  # tanh(w)/s
    l = w - np.log(2.0) + np.log1p(e2)               # ln cosh(w), Re w > 0
    a = h * dxi
    e = l * dxi / (2.0 * s)
    # f = 1 - X h(X^2):  X (s^2 - X^2)^{-1} = [(s - X)^{-1} - (s + X)^{-1}]/2
    # g = X - 2T ln2 - 2T l(X^2):  (s^2 - X^2)^{-1} = [(s - X)^{-1} + (s + X)^{-1}]/(2s)
    poles = np.concatenate([mu + s, mu - np.conj(s)])
    res_f = np.concatenate([0.25j * C * a, -0.25j * C * np.conj(a)])
    res_g = np.concatenate([1j * T * C * e, 1j * T * C * np.conj(e)])
    return {"poles": poles, "res_f": res_f, "res_g": res_g, "f0": 1.0,
            "g0": -mu - 2.0 * T * np.log(2.0), "g1": 1.0}


def evaluate(fit, x, which="f"):
    """The approximant of f ('f'), x f ('ef') or g ('g') at real x."""
    x = np.asarray(x, dtype=np.float64)
    R = 1.0 / (x[..., None] - fit["poles"])
    if which == "f":
        return fit["f0"] + 2.0 * np.real(R @ fit["res_f"])
    if which == "ef":
        # x w/(x - z) = w + w z/(x - z)
        return (fit["f0"] * x + 2.0 * np.real(np.sum(fit["res_f"]))
                + 2.0 * np.real(R @ (fit["res_f"] * fit["poles"])))
    if which == "g":
        return fit["g0"] + fit["g1"] * x + 2.0 * np.real(R @ fit["res_g"])
    raise ValueError(which)


def shifted_solves(H, R, poles, S=None):
    """g_k = (H - z_k S)^{-1} R (S = I when None) for every pole (complex [n, s] each),
    by sparse LU."""
    H = sp.csc_matrix(H, dtype=np.complex128)
    n = H.shape[0]
    M = sp.identity(n, dtype=np.complex128, format="csc") if S is None else sp.csc_matrix(S, dtype=np.complex128)
    Rc = np.asarray(R, dtype=np.complex128)
    return [spla.splu((H - z * M).tocsc()).solve(Rc) for z in poles]


def masked_outer_complex(bsr, X, Y, weights):
    """sum_c w_c X[I-block, c] Y[J-block, c]^T (no conjugation) on every stored block."""
    bd = bsr.block_dim
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    s = X.shape[1]
    Xb = (np.asarray(X) * np.asarray(weights)[None, :]).reshape(-1, bd, s)
    Yb = np.asarray(Y).reshape(-1, bd, s)
    return np.einsum("zac,zbc->zab", Xb[rows], Yb[cols])


def estimate_overlap(bsr, S_values, R, fit, weights=None, density=False):
    """N, E, F with an overlap S on H's pattern (Eq. rational_PQ); optionally the P
    and Q blocks M (.) sum_c w_c (P r_c) r_c^T and M (.) sum_c w_c (Q r_c) r_c^T."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = est.default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    H = bsr.to_scipy().tocsr().astype(np.float64)
    S = bsr.with_values(S_values).to_scipy().tocsr().astype(np.float64)
    z, wf, wg = fit["poles"], fit["res_f"], fit["res_g"]
    gs = shifted_solves(H, R, z, S)
    lu = spla.splu(sp.csc_matrix(S))
    SiR = lu.solve(R)
    SR, HR = S @ R, H @ R
    PR = fit["f0"] * SiR + 2.0 * np.real(sum(wk * gk for wk, gk in zip(wf, gs)))
    FR = (fit["g0"] * np.einsum("ic,ic->c", R, R) + fit["g1"] * np.einsum("ic,ic->c", HR, SiR)
          + 2.0 * np.real(sum(tk * np.einsum("ic,ic->c", SR, gk) for tk, gk in zip(wg, gs))))
    out = {"N": float(w @ np.einsum("ic,ic->c", SR, PR)),
           "E": float(w @ np.einsum("ic,ic->c", HR, PR)),
           "F": float(w @ FR)}
    if density:
        out["density"] = est.masked_outer(bsr, PR, R, w)
        out["density_Q"] = est.masked_outer(bsr, lu.solve(H @ PR), R, w)
    return out


def estimate(bsr, R, fit, weights=None, density=False, gradient=False):
    """N, E, F of the probe estimate with the rational fit; optionally the density
    blocks M (.) sum_c w_c (P r_c) r_c^T and the gradient dF/dH on the pattern."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = est.default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    H = bsr.to_scipy().tocsr().astype(np.float64)
    z, wf, wg = fit["poles"], fit["res_f"], fit["res_g"]
    gs = shifted_solves(H, R, z)
    HR = H @ R
    PR = fit["f0"] * R + 2.0 * np.real(sum(wk * gk for wk, gk in zip(wf, gs)))
    QR = fit["f0"] * HR + 2.0 * np.real(np.sum(wf) * R + sum(wk * zk * gk for wk, zk, gk in zip(wf, z, gs)))
    FR = fit["g0"] * R + fit["g1"] * HR + 2.0 * np.real(sum(tk * gk for tk, gk in zip(wg, gs)))
    out = {
        "N": float(w @ np.einsum("ic,ic->c", R, PR)),
        "E": float(w @ np.einsum("ic,ic->c", R, QR)),
        "F": float(w @ np.einsum("ic,ic->c", R, FR)),
    }
    if density:
        out["density"] = est.masked_outer(bsr, PR, R, w)
    if gradient:
        G = fit["g1"] * est.masked_outer(bsr, R, R, w)
        for tk, gk in zip(wg, gs):
            G = G - 2.0 * np.real(tk * masked_outer_complex(bsr, gk, gk, w))
        out["dFdH"] = G
    return out


def gradient_overlap(bsr, S_values, R, fit, weights=None):
    """(F, G_H, G_S): the probe estimate of F with an overlap (as estimate_overlap) and its
    derivatives with respect to the blocks of H and S, from the rational free-energy
    derivative (Eq. rational_derivative) with the linear part of g added:

      F_c = g0 r.r + g1 r^T H S^{-1} r + 2 Re sum_k tau_k r^T S G_k r,  G_k = (H - z_k S)^{-1},
      dF_c = g1 [r^T dH S^{-1} r - (S^{-1} H r)^T dS S^{-1} r]
             + 2 Re sum_k tau_k [r^T dS g_k + h_k^T (z_k dS - dH) g_k],

    with g_k = G_k r and h_k = G_k S r (G_k^T = G_k for symmetric H and S).  On every stored
    block (I, J):
      G_H[I, J] = sum_c w_c [g1 r[I] (S^{-1} r)[J]^T - 2 Re sum_k tau_k h_k[I] g_k[J]^T],
      G_S[I, J] = sum_c w_c [-g1 (S^{-1} H r)[I] (S^{-1} r)[J]^T
                             + 2 Re sum_k tau_k (r[I] g_k[J]^T + z_k h_k[I] g_k[J]^T)],
    each returned as its symmetric part (G[I, J] + G[J, I]^T)/2 (with S = I, G_H is already
    symmetric and equals estimate's dFdH).  Solves by sparse LU."""
    R = np.asarray(R, dtype=np.float64)
    s = R.shape[1]
    w = est.default_weights(s) if weights is None else np.asarray(weights, dtype=np.float64)
    H = bsr.to_scipy().tocsr().astype(np.float64)
    S = bsr.with_values(S_values).to_scipy().tocsr().astype(np.float64)
    z, wg = fit["poles"], fit["res_g"]
    gs = shifted_solves(H, R, z, S)
    SR = S @ R
    hs = shifted_solves(H, SR, z, S)
    lu = spla.splu(sp.csc_matrix(S))
    SiR = lu.solve(R)
    SiHR = lu.solve(H @ R)
    F = float(w @ (fit["g0"] * np.einsum("ic,ic->c", R, R)
                   + fit["g1"] * np.einsum("ic,ic->c", H @ R, SiR)
                   + 2.0 * np.real(sum(tk * np.einsum("ic,ic->c", SR, gk) for tk, gk in zip(wg, gs)))))
    GH = fit["g1"] * est.masked_outer(bsr, R, SiR, w)
    GS = -fit["g1"] * est.masked_outer(bsr, SiHR, SiR, w)
    for tk, zk, gk, hk in zip(wg, z, gs, hs):
        GH = GH - 2.0 * np.real(tk * masked_outer_complex(bsr, hk, gk, w))
        GS = GS + 2.0 * np.real(tk * (masked_outer_complex(bsr, R.astype(np.complex128), gk, w)
                                      + zk * masked_outer_complex(bsr, hk, gk, w)))
    rows = bsr.block_rows()
    cols = bsr.col_idx.astype(np.int64)
    pos = {(int(i), int(j)): q for q, (i, j) in enumerate(zip(rows, cols))}
    tp = np.array([pos[(int(j), int(i))] for i, j in zip(rows, cols)], dtype=np.int64)
    sym = lambda G: 0.5 * (G + np.transpose(G[tp], (0, 2, 1)))   # noqa: E731
    return F, sym(GH), sym(GS)


def exact(H_dense, fit, S_dense=None):
    """Traces of the rational approximants over the (generalized, with S) eigenvalues
    of a dense symmetric H, P = V diag(f_rat(eps)) V^T and Q = V diag(eps f_rat(eps)) V^T
    (V^T S V = I)."""
    import scipy.linalg as sl
    Hs = np.asarray(H_dense, dtype=np.float64)
    Hs = 0.5 * (Hs + Hs.T)
    if S_dense is None:
        eps, V = np.linalg.eigh(Hs)
    else:
        Ss = np.asarray(S_dense, dtype=np.float64)
        eps, V = sl.eigh(Hs, 0.5 * (Ss + Ss.T))
    f = evaluate(fit, eps, "f")
    return {"N": float(np.sum(f)), "E": float(np.sum(evaluate(fit, eps, "ef"))),
            "F": float(np.sum(evaluate(fit, eps, "g"))), "P": (V * f) @ V.T,
            "Q": (V * (eps * f)) @ V.T}
