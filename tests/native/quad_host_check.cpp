// Host-side check of the plan's quadrature rules (quadrature.cpp): exactness
// of Gauss-Legendre and Gauss-Jacobi on polynomials (closed-form integrals),
// exactness of every Lebedev rule on spherical monomials up to its degree,
// and the antipodal split; Gauss-Laguerre exactness and the composite rule of
// the Debye-Yukawa weight against a fine quadrature after smoothing substitutions.
#include <cmath>
#include <cstdio>
#include <vector>

#include "quadrature.hpp"

static double sphere_monomial(int a, int b, int c) {
  if ((a & 1) || (b & 1) || (c & 1)) return 0.0;
  return 2.0 * std::tgamma((a + 1) / 2.0) * std::tgamma((b + 1) / 2.0) * std::tgamma((c + 1) / 2.0) /
         std::tgamma((a + b + c + 3) / 2.0);
}

int main() {
  int bad = 0;
  // Gauss-Legendre on [0, R]
  for (int n : {1, 4, 16, 32, 64}) {
    std::vector<double> x, w;
    bzq::gauss_legendre(n, 4.0, x, w);
    for (int d = 0; d < std::min(2 * n, 40); ++d) {
      double s = 0;
      for (int i = 0; i < n; ++i) s += w[i] * std::pow(x[i], d);
      const double ex = std::pow(4.0, d + 1) / (d + 1);
      if (std::fabs(s - ex) > 1e-13 * ex) { std::printf("GL n=%d d=%d err=%g\n", n, d, s - ex); ++bad; }
    }
  }
  // Gauss-Jacobi for t^{-s}(1-t)^{-r}
  const double cases[][2] = {{0.5, 0.0}, {0.25, 0.0}, {0.75, 0.0}, {0.0, 0.5}, {0.5, 0.5}, {-1.0, 0.0}, {0.95, 0.0}};
  for (auto& c : cases) {
    for (int n : {8, 32, 64, 128}) {
      std::vector<double> t, w;
      if (!bzq::gauss_jacobi01(n, c[0], c[1], t, w)) { ++bad; continue; }
      // exact moments B(k+1-s, 1-r) by the recurrence B(a+1, b) = B(a, b) a / (a + b)
      long double ex = (long double)std::tgamma(1 - c[0]) * std::tgamma(1 - c[1]) / std::tgamma(2 - c[0] - c[1]);
      for (int k = 0; k < std::min(2 * n, 30); ++k) {
        if (k > 0) ex *= (k - c[0]) / (long double)(k + 1 - c[0] - c[1]);
        double s = 0;
        for (int i = 0; i < n; ++i) s += w[i] * std::pow(t[i], k);
        if (std::fabs(s - ex) > 4e-15 * std::fmax(1.0, ex)) {
          std::printf("GJ s=%g r=%g n=%d k=%d err=%g\n", c[0], c[1], n, k, s - ex);
          ++bad;
        }
      }
    }
  }
  // Lebedev exactness and antipodal halves
  const int sizes[][2] = {{6, 3}, {14, 5}, {26, 7}, {38, 9}, {50, 11}, {74, 13}, {86, 15}, {110, 17},
                          {146, 19}, {170, 21}, {194, 23}, {230, 25}, {266, 27}, {302, 29}, {350, 31}};
  for (auto& sd : sizes) {
    std::vector<double> r, half;
    if (!bzq::lebedev_rule(sd[0], r)) { ++bad; continue; }
    for (int a = 0; a <= sd[1]; ++a)
      for (int b = 0; a + b <= sd[1]; ++b)
        for (int c = 0; a + b + c <= sd[1]; ++c) {
          double s = 0;
          for (int j = 0; j < sd[0]; ++j)
            s += r[4 * j + 3] * std::pow(r[4 * j], a) * std::pow(r[4 * j + 1], b) * std::pow(r[4 * j + 2], c);
          if (std::fabs(s - sphere_monomial(a, b, c)) > 1e-13) {
            std::printf("Lebedev M=%d (%d,%d,%d) err=%g\n", sd[0], a, b, c, s - sphere_monomial(a, b, c));
            ++bad;
          }
        }
    if (bzq::lebedev_half(r, half) != sd[0] / 2) { std::printf("half M=%d\n", sd[0]); ++bad; }
  }
  std::vector<double> r;
  if (bzq::lebedev_rule(37, r)) ++bad;
  // Gauss-Laguerre: exact for u^k, k < 2n (\int e^{-u} u^k du = k!)
  for (int n : {8, 20, 32}) {
    std::vector<long double> u, w;
    bzq::gauss_laguerre(n, u, w);
    long double fact = 1;
    for (int k = 0; k < 2 * n && k < 40; ++k) {
      if (k > 0) fact *= k;
      long double sum = 0;
      for (int i = 0; i < n; ++i) sum += w[i] * powl(u[i], k);
      if (fabsl(sum - fact) > 1e-15L * fact) { std::printf("Laguerre n=%d k=%d err=%Lg\n", n, k, (sum - fact) / fact); ++bad; }
    }
  }
  // Debye rule: nodes in [t_c, 1), positive weights, and \int_0^1 w(t) g(t) dt for
  // g = 1, t, t^2 against a fine quadrature after t = x^4 / 4 on [0, 1/4] and
  // t = 1 - 3 y^2 / 4 on [1/4, 1] (both integrands smooth there)
  for (double tcut : {0.0, 0.3141592653589793}) {
    std::vector<double> t, w;
    if (!bzq::debye_rule(tcut, t, w)) { ++bad; continue; }
    const double tc = std::pow(std::sin(0.5 * tcut), 2);
    for (size_t i = 0; i < t.size(); ++i)
      if (!(t[i] >= tc * (1 - 1e-15) && t[i] < 1.0 && w[i] > 0)) { std::printf("debye node %zu\n", i); ++bad; break; }
    std::vector<double> gx, gw;
    bzq::gauss_legendre(400, 1.0, gx, gw);
    for (int k = 0; k < 3; ++k) {
      long double ref = 0;
      for (int i = 0; i < 400; ++i) {
        const long double x = gx[i], ta = x * x * x * x / 4;        // [0, 1/4]
        if (ta >= tc) ref += gw[i] * (-logl(2 * sqrtl(ta))) / sqrtl(1 - ta) * powl(ta, k) * x * x * x;
        const long double y = gx[i], tb = 1 - 0.75L * y * y;          // [1/4, 1]
        ref += gw[i] * logl(2 * sqrtl(tb)) * powl(tb, k) * 1.5L / sqrtl(0.75L);
      }
      if (tcut > 0) {   // the part of [0, 1/4] below t_c is excluded; redo [t_c, 1/4] directly
        ref = 0;
        for (int i = 0; i < 400; ++i) {
          const long double ta = tc + (0.25L - tc) * gx[i];
          ref += gw[i] * (0.25L - tc) * (-logl(2 * sqrtl(ta))) / sqrtl(1 - ta) * powl(ta, k);
          const long double y = gx[i], tb = 1 - 0.75L * y * y;
          ref += gw[i] * logl(2 * sqrtl(tb)) * powl(tb, k) * 1.5L / sqrtl(0.75L);
        }
      }
      long double sum = 0;
      for (size_t i = 0; i < t.size(); ++i) sum += w[i] * powl((long double)t[i], k);
      if (fabsl(sum - ref) > 1e-13L * fabsl(ref)) {
        std::printf("debye rule theta_cut=%g k=%d: %.18Lg vs %.18Lg\n", tcut, k, sum, ref);
        ++bad;
      }
    }
  }
  std::printf("quadrature host check: %d failures\n", bad);
  return bad ? 1 : 0;
}
