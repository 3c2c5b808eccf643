// Kernel functions kappa(x, y; theta) of Table "Kernel functions", shared by the host offline
// stage and its GPU kernel-tensor generation (one implementation, compiled for both sides).
// The Matern kernel with free nu needs the modified Bessel function K_nu; the parts of it that
// depend on nu only (BesselOrder) are computed on the host (special.cpp) and passed in.
//
// K_nu is reduced to K_mu, K_{mu+1} with |mu| <= 1/2, nu = mu + m, and raised by the
// recurrence K_{a+1}(x) = K_{a-1}(x) + (2 a / x) K_a(x), which is stable upward.
//   x <= 2: Temme's series (N. M. Temme, J. Comput. Phys. 19, 1975):
//     K_mu = sum_k c_k f_k,  K_{mu+1} = (2 / x) sum_k c_k (p_k - k f_k),  c_k = (x^2 / 4)^k / k!,
//     f_k = (k f_{k-1} + p_{k-1} + q_{k-1}) / (k^2 - mu^2),  p_k = p_{k-1} / (k - mu),
//     q_k = q_{k-1} / (k + mu),  p_0 = (x / 2)^-mu Gamma(1 + mu) / 2,  q_0 = (x / 2)^mu Gamma(1 - mu) / 2,
//     f_0 = (mu pi / sin(mu pi)) (cosh(s) G1(mu) + (sinh(s) / s) ln(2 / x) G2(mu)),  s = mu ln(2 / x),
//     G1 = (1 / Gamma(1 - mu) - 1 / Gamma(1 + mu)) / (2 mu),  G2 = (1 / Gamma(1 - mu) + 1 / Gamma(1 + mu)) / 2.
//   x > 2: K_mu(x) = sqrt(pi) (2 x)^mu e^-x U(mu + 1/2, 2 mu + 1, 2 x) (Kummer's U).  In n,
//     y_n = U(mu + 1/2 + n, 2 mu + 1, 2 x) is the minimal solution of
//       y_{n-1} - 2 (n + x) y_n + ((n + 1/2)^2 - mu^2) y_{n+1} = 0,
//     obtained by backward recurrence from a far start (Miller's algorithm) and normalised
//     with sum_n C_n y_n / y_0 = sqrt(pi / (2 x)) e^-x / K_mu(x), C_0 = 1,
//     C_n = C_{n-1} ((n - 1/2)^2 - mu^2) / n (the normalisation of Steed's method,
//     I. J. Thompson and A. R. Barnett, J. Comput. Phys. 64, 1986); then
//     K_{mu+1} = K_mu (mu + x + 1/2 + (mu^2 - 1/4) y_1 / y_0) / x.
// Both branches return e^x K (scaled) so that the kernel never under- or overflows early.
#pragma once

#include <cmath>

#include "ph.h"

#if defined(__HIPCC__)
#define PH_HD __host__ __device__
#else
#define PH_HD
#endif

namespace ph {

// nu-only constants of K_nu: nu = mu + m with mu in [-1/2, 1/2), G1(mu), G2(mu), ln Gamma(nu)
struct BesselOrder {
  double mu, g1, g2, lgam;
  int m;
};

// e^x K_mu(x), e^x K_{mu+1}(x), |mu| <= 1/2, 0 < x <= 2 (Temme's series)
PH_HD inline void bessel_k_small(double mu, double g1, double g2, double x, double& k0, double& k1) {
  const double pi = 3.14159265358979323846;
  const double gp = 1 / (g2 - mu * g1), gm = 1 / (g2 + mu * g1);   // Gamma(1 + mu), Gamma(1 - mu)
  const double L = std::log(2 / x), s = mu * L;
  const double fac = mu == 0 ? 1.0 : mu * pi / std::sin(mu * pi);
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
PH_HD inline void bessel_k_large(double mu, double x, double& k0, double& k1) {
  const double pi = 3.14159265358979323846;
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
  k0 = std::sqrt(pi / (2 * x)) / S;
  k1 = k0 * (mu + x + 0.5 + (mu * mu - 0.25) * y[1] / y[0]) / x;
}

// e^x K_nu(x) for the order described by o, x > 0
PH_HD inline double bessel_k_scaled_o(const BesselOrder& o, double x) {
  double a, b;
  if (x <= 2) bessel_k_small(o.mu, o.g1, o.g2, x, a, b);
  else bessel_k_large(o.mu, x, a, b);
  for (int j = 0; j < o.m; ++j) {   // a = K_{mu+j}, b = K_{mu+j+1}
    const double c = a + 2 * (o.mu + j + 1) / x * b;
    a = b;
    b = c;
  }
  return a;
}

// 2^(1 - nu) / Gamma(nu) z^nu K_nu(z), z = sqrt(2 nu) r / lambda; 1 at r = 0
PH_HD inline double matern_o(double r, double lambda, double nu, const BesselOrder& o) {
  if (r == 0) return 1.0;
  const double z = std::sqrt(2 * nu) * r / lambda;
  if (z > 745) return 0.0;
  const double lg = (1 - nu) * 0.69314718055994530942 - o.lgam + nu * std::log(z) - z;
  return std::exp(lg) * bessel_k_scaled_o(o, z);
}

// kappa(x, y; theta) for the kernels of ph_kernel; o describes nu = theta[1] for the Matern
// kernel (unused otherwise)
PH_HD inline double kernel_eval(ph_kernel k, int d, const double* x, const double* y, const double* th,
                                const BesselOrder& o) {
  double r2 = 0;
  for (int i = 0; i < d; ++i) r2 += (x[i] - y[i]) * (x[i] - y[i]);
  switch (k) {
    case PH_KERNEL_GAUSSIAN:
      return std::exp(-r2 / (2.0 * th[0] * th[0]));
    case PH_KERNEL_MATERN32: {
      const double s = std::sqrt(3.0) * std::sqrt(r2) / th[0];
      return (1.0 + s) * std::exp(-s);
    }
    case PH_KERNEL_MATERN12:
      return std::exp(-std::sqrt(r2) / th[0]);
    case PH_KERNEL_ANISO_GAUSSIAN: {
      double e = 0;
      for (int i = 0; i < d; ++i) e += (x[i] - y[i]) * (x[i] - y[i]) / (2.0 * th[i] * th[i]);
      return std::exp(-e);
    }
    case PH_KERNEL_POLY_TEST:
      return th[0] * th[0] * r2 + th[0];
    case PH_KERNEL_POLY2_TEST:
      return th[0] * r2 + th[1] * th[1];
    case PH_KERNEL_MATERN:
      return matern_o(std::sqrt(r2), th[0], th[1], o);
  }
  return 0.0;
}

}  // namespace ph
