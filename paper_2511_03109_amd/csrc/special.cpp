// Host side of the modified Bessel function K_nu (Matern kernel with free nu, Table "Kernel
// functions"): the constants that depend on the order only (BesselOrder: mu, G1(mu), G2(mu),
// ln Gamma(nu)), and the host entry points.  The series and recurrences themselves are in
// kernel_fn.hpp, shared with the GPU kernel-tensor generation.
// G1 and G2 come from the Taylor series of ln Gamma(1 + z) (coefficients zeta(k) / k), split into
// its odd and even parts, so that the removable singularity of G1 at mu = 0 costs no accuracy.
// Measured against adaptive quadrature of K_nu(x) = int_0^inf exp(-x cosh t) cosh(nu t) dt
// (itself good to about 1e-14): agreement within 1.4e-14 relative for 0.5 <= nu <= 3,
// 1e-8 <= x <= 600.  The offline stage evaluates the kernel at a few nu (the Chebyshev nodes of
// Theta), so the order constants are kept per thread for the last 16 orders seen.
#include <cmath>
#include <cstdint>

#include "kernel_fn.hpp"
#include "ph_host.hpp"

namespace ph {
namespace {

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

// per-order constants, cached per thread
struct OrderConst {
  double nu = -1;
  BesselOrder o{};
};

const BesselOrder& order_const(double nu) {
  thread_local OrderConst cache[16];
  thread_local int next = 0;
  for (const OrderConst& c : cache)
    if (c.nu == nu) return c.o;
  OrderConst& c = cache[next];
  next = (next + 1) % 16;
  c.nu = nu;
  c.o.m = (int)std::floor(nu + 0.5);
  c.o.mu = nu - c.o.m;
  gamma12(c.o.mu, c.o.g1, c.o.g2);
  c.o.lgam = std::lgamma(nu);
  return c.o;
}

}  // namespace

BesselOrder bessel_order(double nu) { return order_const(nu); }

double bessel_k_scaled(double nu, double x) { return bessel_k_scaled_o(order_const(nu), x); }

double matern_value(double r, double lambda, double nu) { return matern_o(r, lambda, nu, order_const(nu)); }

}  // namespace ph
