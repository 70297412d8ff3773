// Pole fit of the rational expansion (paper: Rational approximation, Eq.
// rational_fit), host code only.
//
// The paper's best fit is numerical and its poles are not printed; the fit here
// is the analytical kind it names for a finite spectral interval, usable for
// both the Fermi function f and the free-energy function g: the trapezoid rule
// of a Cauchy integral on a conformal map of an annulus (Hale, Higham and
// Trefethen 2008, first method, functions analytic off (-inf, 0]).  With
// X = x - mu the even parts of f and g are functions of u = X^2,
//   f = 1 - X h(u),            h(u) = tanh(sqrt(u)/(2T)) / sqrt(u),
//   g = X - 2T ln 2 - 2T l(u), l(u) = ln cosh(sqrt(u)/(2T)),
// analytic off u <= -(pi T)^2.  In xi = u + (pi T)^2 the rule applies on
// [m, M] = [(pi T)^2, D^2 + (pi T)^2], D = max |e - mu| over the interval.  Node
// xi_j gives s_j = sqrt(xi_j - m) and the poles mu + s_j and mu - conj(s_j).
//
// Jacobi's elliptic functions come from the arithmetic-geometric mean
// (Abramowitz & Stegun 16.4 and 17.6), at complex argument through Jacobi's
// imaginary transformation and the addition theorems.
#include <cmath>
#include <complex>
#include <vector>

#include "rfo.h"

namespace {

using cd = std::complex<double>;

// K for modulus k = sqrt(1 - kp^2), given the complementary modulus kp:
// K = pi / (2 AGM(1, kp)).
double ellip_k_from_kp(double kp) {
  double a = 1.0, b = kp;
  for (int i = 0; i < 64 && std::fabs(a - b) > 1e-16 * a; ++i) {
    const double an = 0.5 * (a + b);
    b = std::sqrt(a * b);
    a = an;
  }
  return M_PI / (a + b);
}

// sn, cn, dn of real u for modulus k, complementary modulus kp (k^2 + kp^2 = 1),
// by the descending AGM scale: a_0 = 1, b_0 = kp, c_0 = k; phi_N = 2^N a_N u,
// phi_{n-1} = (phi_n + asin(c_n sin(phi_n) / a_n)) / 2.
void jacobi_real(double u, double k, double kp, double &sn, double &cn, double &dn) {
  double a[40], c[40];
  a[0] = 1.0;
  double b = kp;
  c[0] = k;
  int n = 0;
  while (n < 38 && std::fabs(c[n]) > 1e-17) {
    const double an = 0.5 * (a[n] + b);
    c[n + 1] = 0.5 * (a[n] - b);
    b = std::sqrt(a[n] * b);
    a[n + 1] = an;
    ++n;
  }
  double phi = std::ldexp(a[n] * u, n);
  double phi_prev = phi;
  for (int i = n; i >= 1; --i) {
    phi_prev = phi;
    phi = 0.5 * (phi + std::asin(c[i] * std::sin(phi) / a[i]));
  }
  sn = std::sin(phi);
  cn = std::cos(phi);
  dn = n > 0 ? cn / std::cos(phi_prev - phi) : 1.0;
}

// sn, cn, dn at x + i y for modulus k (kp complementary).
void jacobi_complex(double x, double y, double k, double kp, cd &sn, cd &cn, cd &dn) {
  double s, c, d, s1, c1, d1;
  jacobi_real(x, k, kp, s, c, d);
  jacobi_real(y, kp, k, s1, c1, d1);  // complementary modulus
  const cd sb(0.0, s1 / c1);          // sn(i y) = i sc(y, kp)
  const double cb = 1.0 / c1, db = d1 / c1;
  const double m = k * k;
  const cd den = 1.0 - m * s * s * sb * sb;
  sn = (s * cb * db + sb * c * d) / den;
  cn = (c * cb - s * d * sb * db) / den;
  dn = (d * db - m * s * c * sb * cb) / den;
}

}  // namespace

extern "C" int rfo_rational_fit(int n_nodes, double T, double mu, double e_min, double e_max,
                                double *poles, double *res_f, double *res_g, double *poly) {
  if (n_nodes < 1 || n_nodes > 1024 || !poles || !res_f || !res_g || !poly) return RFO_E_INVALID;
  if (!(T > 0.0) || !std::isfinite(T) || !std::isfinite(mu) || !std::isfinite(e_min) ||
      !std::isfinite(e_max) || !(e_max > e_min))
    return RFO_E_INVALID;
  const double D = std::max(std::fabs(e_min - mu), std::fabs(e_max - mu));
  const double m = (M_PI * T) * (M_PI * T);
  const double M = D * D + m;
  const double q = std::sqrt(M / m);
  if (!(q > 1.0) || !std::isfinite(q)) return RFO_E_INVALID;
  const double k = (q - 1.0) / (q + 1.0);
  const double kp = 2.0 * std::sqrt(q) / (q + 1.0);  // sqrt(1 - k^2) without cancellation
  const double K = ellip_k_from_kp(kp), Kp = ellip_k_from_kp(k);
  const double c = std::sqrt(m * M);
  const double C = 4.0 * K * c / (M_PI * n_nodes * k);
  const int n = n_nodes;
  for (int j = 0; j < n; ++j) {
    const double t = -K + (j + 0.5) * (2.0 * K / n);
    cd sn, cn, dn;
    jacobi_complex(t, 0.5 * Kp, k, kp, sn, cn, dn);
    const cd xi = c * (1.0 / k + sn) / (1.0 / k - sn);
    const cd dxi = cn * dn / ((1.0 / k - sn) * (1.0 / k - sn));
    const cd s = std::sqrt(xi - m);
    const cd w = s / (2.0 * T);
    const cd e2 = std::exp(-2.0 * w);
    const cd h = (1.0 - e2) / (1.0 + e2) / s;
    const cd l = w - std::log(2.0) + std::log(1.0 + e2);
    const cd a = h * dxi;
    const cd e = l * dxi / (2.0 * s);
    const cd I(0.0, 1.0);
    const cd zp = mu + s, zm = mu - std::conj(s);
    const cd fp = 0.25 * I * C * a, fm = -0.25 * I * C * std::conj(a);
    const cd gp = I * T * C * e, gm = I * T * C * std::conj(e);
    const cd vals[6] = {zp, zm, fp, fm, gp, gm};
    for (const cd &v : vals)
      if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return RFO_E_NUMERIC;
    poles[2 * j] = zp.real();
    poles[2 * j + 1] = zp.imag();
    poles[2 * (n + j)] = zm.real();
    poles[2 * (n + j) + 1] = zm.imag();
    res_f[2 * j] = fp.real();
    res_f[2 * j + 1] = fp.imag();
    res_f[2 * (n + j)] = fm.real();
    res_f[2 * (n + j) + 1] = fm.imag();
    res_g[2 * j] = gp.real();
    res_g[2 * j + 1] = gp.imag();
    res_g[2 * (n + j)] = gm.real();
    res_g[2 * (n + j) + 1] = gm.imag();
  }
  poly[0] = 1.0;                          // f0
  poly[1] = -mu - 2.0 * T * std::log(2.0);  // g0
  poly[2] = 1.0;                          // g1
  return RFO_OK;
}
