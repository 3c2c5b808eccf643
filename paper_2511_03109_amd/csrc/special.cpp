// Modified Bessel function of the second kind K_nu(x) (real order nu >= 0, x > 0) and the
// Matern kernel built on it (Table "Kernel functions": MN with parameters (lambda, nu)).
//
// K_nu is reduced to K_mu, K_{mu+1} with |mu| <= 1/2, nu = mu + m, and raised by the
// recurrence K_{a+1}(x) = K_{a-1}(x) + (2 a / x) K_a(x), which is stable upward.
//   x <= 2: Temme's series (N. M. Temme, J. Comput. Phys. 19, 1975):
//     K_mu = sum_k c_k f_k,  K_{mu+1} = (2 / x) sum_k c_k (p_k - k f_k),  c_k = (x^2 / 4)^k / k!,
//     f_k = (k f_{k-1} + p_{k-1} + q_{k-1}) / (k^2 - mu^2),  p_k = p_{k-1} / (k - mu),
//     q_k = q_{k-1} / (k + mu),  p_0 = (x / 2)^-mu Gamma(1 + mu) / 2,  q_0 = (x / 2)^mu Gamma(1 - mu) / 2,
//     f_0 = (mu pi / sin(mu pi)) (cosh(s) G1(mu) + (sinh(s) / s) ln(2 / x) G2(mu)),  s = mu ln(2 / x),
//     G1 = (1 / Gamma(1 - mu) - 1 / Gamma(1 + mu)) / (2 mu),  G2 = (1 / Gamma(1 - mu) + 1 / Gamma(1 + mu)) / 2.
//     G1 and G2 come from the Taylor series of ln Gamma(1 + z) (coefficients zeta(k) / k),
//     split into its odd and even parts, so that the removable singularity of G1 at mu = 0
//     costs no accuracy.
//   x > 2: K_mu(x) = sqrt(pi) (2 x)^mu e^-x U(mu + 1/2, 2 mu + 1, 2 x) (Kummer's U).  In n,
//     y_n = U(mu + 1/2 + n, 2 mu + 1, 2 x) is the minimal solution of
//       y_{n-1} - 2 (n + x) y_n + ((n + 1/2)^2 - mu^2) y_{n+1} = 0,
//     obtained by backward recurrence from a far start (Miller's algorithm) and normalised
//     with sum_n C_n y_n / y_0 = sqrt(pi / (2 x)) e^-x / K_mu(x), C_0 = 1,
//     C_n = C_{n-1} ((n - 1/2)^2 - mu^2) / n (the normalisation of Steed's method,
//     I. J. Thompson and A. R. Barnett, J. Comput. Phys. 64, 1986); then
//     K_{mu+1} = K_mu (mu + x + 1/2 + (mu^2 - 1/4) y_1 / y_0) / x.
// Both branches return e^x K (scaled) so that the kernel never under- or overflows early.
// Measured against adaptive quadrature of K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
// (itself good to about 1e-14): agreement within 1.4e-14 relative for 0.5 <= nu <= 3,
// 1e-8 <= x <= 600.  G1, G2 and ln Gamma(nu) depend on nu only: the offline stage evaluates
// the kernel at a few nu (the Chebyshev nodes of Theta), so they are kept per thread for
// the last 16 orders seen.
#include <cmath>
#include <cstdint>

#include "ph_host.hpp"

namespace ph {
namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr int kZetaMax = 60;

// zeta(k), k = 2 .. kZetaMax: the first 15 terms summed, the rest by Euler-Maclaurin with
// Bernoulli numbers B_2 .. B_16 (remainder below 1e-19 for k >= 2)
struct ZetaTable {
  double z[kZetaMax + 1];
  ZetaTable() {
    const double bern[8] = {1.0 / 6, -1.0 / 30, 1.0 / 42, -1.0 / 30, 5.0 / 66, -691.0 / 2730, 7.0 / 6, -3617.0 / 510};
    const int N = 16;
    for (int k = 2; k <= kZetaMax; ++k) {
      long double s = 0;
      for (int n = N - 1; n >= 1; --n) s += std::pow((long double)n, (long double)-k);
      long double tail = std::pow((long double)N, (long double)(1 - k)) / (k - 1) +
                         0.5L * std::pow((long double)N, (long double)-k);
      long double fact = 1, rising = 1;
      for (int j = 1; j <= 8; ++j) {
        rising = j == 1 ? (long double)k : rising * (k + 2 * j - 3) * (k + 2 * j - 2);
        fact *= (long double)(2 * j - 1) * (2 * j);
        tail += bern[j - 1] / fact * rising * std::pow((long double)N, (long double)(-k - 2 * j + 1));
      }
      z[k] = (double)(s + tail);
    }
  }
};

const ZetaTable& zeta_table() {
  static const ZetaTable t;
  return t;
}

// G1(mu), G2(mu) for |mu| <= 1/2.  1 / Gamma(1 + z) = exp(E(z)),
// E(z) = gamma z + sum_{k >= 2} (-1)^{k+1} zeta(k) z^k / k = O(z) + V(z) (odd + even part);
// G1 = -e^V sinh(O) / mu, G2 = e^V cosh(O).
void gamma12(double mu, double& g1, double& g2) {
  const double* z = zeta_table().z;
  double o = kEulerGamma;   // O(mu) / mu
  double v = 0;
  double p = 1;             // mu^(k-1)
  for (int k = 2; k <= kZetaMax; ++k) {
    p *= mu;
    if (k & 1) o += z[k] * p / k;
    else v -= z[k] * p * mu / k;
  }
  const double O = mu * o;
  const double shc = std::fabs(O) < 1e-4 ? 1 + O * O / 6 * (1 + O * O / 20) : std::sinh(O) / O;
  const double ev = std::exp(v);
  g1 = -ev * o * shc;
  g2 = ev * std::cosh(O);
}

// per-order constants: mu, G1(mu), G2(mu), ln Gamma(nu)
struct OrderConst {
  double nu = -1, mu = 0, g1 = 0, g2 = 0, lgam = 0;
  int m = 0;   // nu = mu + m
};

const OrderConst& order_const(double nu) {
  thread_local OrderConst cache[16];
  thread_local int next = 0;
  for (const OrderConst& c : cache)
    if (c.nu == nu) return c;
  OrderConst& c = cache[next];
  next = (next + 1) % 16;
  c.nu = nu;
  c.m = (int)std::floor(nu + 0.5);
  c.mu = nu - c.m;
  gamma12(c.mu, c.g1, c.g2);
  c.lgam = std::lgamma(nu);
  return c;
}

// e^x K_mu(x), e^x K_{mu+1}(x), |mu| <= 1/2, 0 < x <= 2 (Temme's series)
void k_small(double mu, double g1, double g2, double x, double& k0, double& k1) {
  const double gp = 1 / (g2 - mu * g1), gm = 1 / (g2 + mu * g1);   // Gamma(1 + mu), Gamma(1 - mu)
  const double L = std::log(2 / x), s = mu * L;
  const double fac = mu == 0 ? 1.0 : mu * kPi / std::sin(mu * kPi);
  const double shs = s == 0 ? 1.0 : std::sinh(s) / s;
  double f = fac * (std::cosh(s) * g1 + shs * L * g2);
  double p = 0.5 * std::exp(s) * gp, q = 0.5 * std::exp(-s) * gm;
  double c = 1, s0 = f, s1 = p;
  const double x2 = 0.25 * x * x;
  for (int k = 1; k < 200; ++k) {
    f = (k * f + p + q) / (k * (double)k - mu * mu);
    p /= k - mu;
    q /= k + mu;
    c *= x2 / k;
    const double a = c * f, b = c * (p - k * f);
    s0 += a;
    s1 += b;
    if (std::fabs(a) < 1e-17 * std::fabs(s0) && std::fabs(b) < 1e-17 * std::fabs(s1)) break;
  }
  const double ex = std::exp(x);
  k0 = s0 * ex;
  k1 = s1 * 2 / x * ex;
}

// e^x K_mu(x), e^x K_{mu+1}(x), |mu| <= 1/2, x > 2 (minimal solution by backward recurrence)
void k_large(double mu, double x, double& k0, double& k1) {
  const int N = x < 4 ? 100 : 60;
  double y[102];
  y[N + 1] = 0;
  y[N] = 1e-300;
  for (int n = N; n >= 1; --n) {
    y[n - 1] = 2 * (n + x) * y[n] - ((n + 0.5) * (n + 0.5) - mu * mu) * y[n + 1];
    if (std::fabs(y[n - 1]) > 1e250)   // rescale everything computed so far
      for (int m = n - 1; m <= N; ++m) y[m] *= 1e-250;
  }
  double C = 1, S = y[0];
  for (int n = 1; n <= N; ++n) {
    C *= ((n - 0.5) * (n - 0.5) - mu * mu) / n;
    S += C * y[n];
  }
  S /= y[0];
  k0 = std::sqrt(kPi / (2 * x)) / S;
  k1 = k0 * (mu + x + 0.5 + (mu * mu - 0.25) * y[1] / y[0]) / x;
}

}  // namespace

double bessel_k_scaled(double nu, double x) {
  const OrderConst& oc = order_const(nu);
  const double mu = oc.mu;          // in [-1/2, 1/2)
  double a, b;
  if (x <= 2) k_small(mu, oc.g1, oc.g2, x, a, b);
  else k_large(mu, x, a, b);
  for (int j = 0; j < oc.m; ++j) {   // a = K_{mu+j}, b = K_{mu+j+1}
    const double c = a + 2 * (mu + j + 1) / x * b;
    a = b;
    b = c;
  }
  return a;
}

double matern_value(double r, double lambda, double nu) {
  if (r == 0) return 1.0;
  const double z = std::sqrt(2 * nu) * r / lambda;
  if (z > 745) return 0.0;
  // 2^(1 - nu) / Gamma(nu) z^nu K_nu(z), with K_nu(z) = e^-z (e^z K_nu(z))
  const double lg = (1 - nu) * std::log(2.0) - order_const(nu).lgam + nu * std::log(z) - z;
  return std::exp(lg) * bessel_k_scaled(nu, z);
}

}  // namespace ph
