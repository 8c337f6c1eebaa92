// Host-side check of the series of the angular weight (funk_hecke.cpp):
// * spherical Bessel functions against their closed forms for l <= 3 and
//   against the (stable) upward recurrence for l < x;
// * mu_l for constant b (eq. cutoff3D: mu_l = -4 pi c for every l >= 2) and
//   mu_2 for b = c t^{-1-s} (1-t)^{-r} against the Beta-function closed form;
// * the even-Legendre recurrence against the Legendre three-term recurrence,
//   and its Chebyshev connection matrix against direct evaluation;
// * the whole series for constant b against eq. cutoff3D,
//   Re(e^{-ix} F) = 4 pi c (sin r / r - cos x).
#include <cmath>
#include <cstdio>
#include <vector>

#include "funk_hecke.hpp"

static long double legendre(int l, long double t) {
  long double p0 = 1.0L, p1 = t;
  if (l == 0) return p0;
  for (int n = 1; n < l; ++n) {
    const long double p2 = ((2 * n + 1) * t * p1 - n * p0) / (n + 1);
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

int main() {
  int bad = 0;
  const long double pi = 3.141592653589793238462643383279502884L;
  // spherical Bessel
  for (long double x : {0.01L, 0.3L, 1.0L, 3.14159L, 7.5L, 22.0L, 41.3L, 63.0L}) {
    std::vector<long double> j;
    bzq::fh_sph_bessel(120, x, j);
    const long double s = sinl(x), c = cosl(x);
    const long double ex[4] = {s / x, s / (x * x) - c / x, (3 / (x * x) - 1) * s / x - 3 * c / (x * x),
                               (15 / (x * x * x) - 6 / x) * s / x - (15 / (x * x) - 1) * c / x};
    long double exs[4];
    if (x < 0.1L) {
      // the closed forms cancel for small x: j_l = x^l / (2l+1)!! (1 - x^2 / (2 (2l+3)) + x^4 / (8 (2l+3)(2l+5)))
      long double df = 1.0L;
      for (int l = 0; l < 4; ++l) {
        df *= (2 * l + 1);
        exs[l] = powl(x, l) / df * (1 - x * x / (2 * (2 * l + 3)) + powl(x, 4) / (8 * (2 * l + 3) * (2 * l + 5)));
      }
    } else {
      for (int l = 0; l < 4; ++l) exs[l] = ex[l];
    }
    for (int l = 0; l < 4; ++l)
      if (fabsl(j[l] - exs[l]) > 1e-15L * (x < 0.1L ? fabsl(exs[l]) : 10.0L)) {
        std::printf("j_%d(%Lg) = %.18Lg vs %.18Lg\n", l, x, j[l], exs[l]);
        ++bad;
      }
    // upward recurrence is stable for l < x
    long double a = ex[0], b = ex[1];
    for (int l = 1; l + 1 < (int)x && l < 120; ++l) {
      const long double nb = (2 * l + 1) / x * b - a;
      a = b;
      b = nb;
      if (fabsl(j[l + 1] - b) > 1e-13L) {
        std::printf("j_%d(%Lg) = %.18Lg vs upward %.18Lg\n", l + 1, x, j[l + 1], b);
        ++bad;
        break;
      }
    }
  }
  // mu_l, constant b = c (s = -1, r = 0): lambda_l = 0 for l >= 1
  {
    std::vector<long double> mu;
    const double c = 1.0 / (4.0 * (double)pi);
    if (!bzq::fh_moments(100, c, -1.0, 0.0, mu)) ++bad;
    for (int m = 1; m <= 50; ++m)
      if (fabsl(mu[m] + 1.0L) > 1e-14L) { std::printf("cutoff mu_%d = %.18Lg\n", 2 * m, mu[m]); ++bad; }
  }
  // mu_2 = 4 pi c \int t^{-s} (1-t)^{-r} (-6 (1 - t)) dt = -24 pi c B(1-s, 2-r)
  const double cases[][3] = {{0.02, 0.25, 0.0}, {0.01, 0.5, 0.0}, {0.003, 0.75, 0.0}, {0.05, 0.25, 0.5},
                             {0.02, -0.5, 0.0}};
  for (auto& cs : cases) {
    std::vector<long double> mu;
    if (!bzq::fh_moments(40, cs[0], cs[1], cs[2], mu)) { ++bad; continue; }
    const long double B = tgammal(1 - cs[1]) * tgammal(2 - cs[2]) / tgammal(3 - cs[1] - cs[2]);
    const long double ex = -24.0L * pi * cs[0] * B;
    if (fabsl(mu[1] - ex) > 1e-14L * fabsl(ex)) {
      std::printf("mu_2 (s=%g r=%g) = %.18Lg vs %.18Lg\n", cs[1], cs[2], mu[1], ex);
      ++bad;
    }
  }
  // even Legendre recurrence
  {
    for (long double t : {-0.93L, -0.2L, 0.0L, 0.41L, 0.999L}) {
      const long double u = 2 * t * t - 1;
      long double q0 = 0.0L, q1 = 1.0L;
      for (int m = 1; m <= 60; ++m) {
        const long double q2 = (bzq::fh_rec_A(m) * u + bzq::fh_rec_B(m)) * q1 - bzq::fh_rec_C(m) * q0;
        q0 = q1;
        q1 = q2;
        if (fabsl(q1 - legendre(2 * m, t)) > 1e-13L) {
          std::printf("P_%d(%Lg) recurrence %.18Lg vs %.18Lg\n", 2 * m, t, q1, legendre(2 * m, t));
          ++bad;
          break;
        }
      }
    }
  }
  // Chebyshev form: sum_m c_m Q_m(u) = sum_k (M c)_k T_k(u)
  {
    const int mm = 44;
    std::vector<long double> M;
    bzq::fh_cheb_matrix(mm, M);
    std::vector<long double> cc(mm), d(mm, 0.0L);
    for (int m = 0; m < mm; ++m) cc[m] = sinl(1.7L * m + 0.3L) / (1 + m);
    for (int k = 0; k < mm; ++k)
      for (int m = k; m < mm; ++m) d[k] += M[(size_t)k * mm + m] * cc[m];
    for (long double t : {-0.97L, -0.5L, 0.1L, 0.66L, 1.0L}) {
      const long double u = 2 * t * t - 1;
      long double a = 0.0L, b = 0.0L;
      for (int m = 0; m < mm; ++m) a += cc[m] * legendre(2 * m, t);
      for (int k = 0; k < mm; ++k) b += d[k] * cosl(k * acosl(u));
      if (fabsl(a - b) > 1e-15L * 10) { std::printf("chebyshev form t=%Lg: %.18Lg vs %.18Lg\n", t, a, b); ++bad; }
    }
  }
  // the series for constant b against eq. cutoff3D
  {
    const double c = 1.0 / (4.0 * (double)pi);
    for (double r : {0.5, 4.0, 17.0, 38.0, 55.0}) {
      const int lmax = bzq::fh_lmax(r);
      std::vector<long double> mu, j;
      bzq::fh_moments(lmax, c, -1.0, 0.0, mu);
      bzq::fh_sph_bessel(lmax, r, j);
      for (double t : {-0.9, -0.3, 0.05, 0.6, 1.0}) {
        long double sum = 0.0L;
        for (int l = 0; l <= lmax; l += 2)
          sum += (2 * l + 1) * (((l / 2) & 1) ? -1.0L : 1.0L) * mu[l / 2] * j[l] * legendre(l, t);
        const long double ex = sinl(r) / r - cosl(r * t);
        if (fabsl(sum - ex) > 1e-13L) {
          std::printf("series r=%g t=%g: %.18Lg vs %.18Lg\n", r, t, sum, ex);
          ++bad;
        }
      }
    }
  }
  std::printf("series host check: %d failures\n", bad);
  return bad ? 1 : 0;
}
