// Series coefficients of the angular weight (see funk_hecke.hpp).
#include "funk_hecke.hpp"

#include <cmath>

#include "quadrature.hpp"

namespace bzq {

int fh_lmax(double r) {
  // l - r grows like r^{1/3}: measured margins for 1e-14 are 25, 30, 35, 40 at r = 10, 20, 40, 55
  int l = (int)std::ceil(r + 8.0 * std::cbrt(r) + 12.0);
  return l + (l & 1);
}

bool fh_moments(int lmax, double c, double s, double r, std::vector<long double>& mu) {
  const int n = lmax / 2 + 8;
  std::vector<double> t, w;
  if (!gauss_jacobi01(n, s, r, t, w)) return false;
  mu.assign(lmax / 2 + 1, 0.0L);
  const long double fourpic = 4.0L * 3.141592653589793238462643383279502884L * c;
  for (int i = 0; i < n; ++i) {
    // E_l = (P_l(1 - 2t) - 1) / t by the Legendre recurrence written for the
    // difference: E_0 = 0, E_1 = -2, (l+1) E_{l+1} = (2l+1)(u E_l - 2) - l E_{l-1}
    const long double ti = t[i], u = 1.0L - 2.0L * ti;
    long double e0 = 0.0L, e1 = -2.0L;
    for (int l = 1; l < lmax; ++l) {
      const long double e2 = ((2 * l + 1) * (u * e1 - 2.0L) - l * e0) / (l + 1);
      e0 = e1;
      e1 = e2;
      if ((l + 1) % 2 == 0) mu[(l + 1) / 2] += (long double)w[i] * e1;
    }
  }
  for (auto& m : mu) m *= fourpic;
  mu[0] = 0.0L;
  return true;
}

void fh_sph_bessel(int lmax, long double x, std::vector<long double>& j) {
  j.assign(lmax + 1, 0.0L);
  if (x == 0.0L) {
    j[0] = 1.0L;
    return;
  }
  const int start = lmax + 40 + (int)(2.0L * x);
  long double jp = 0.0L, jc = 1e-300L, norm = 0.0L;
  std::vector<long double> tmp(lmax + 1, 0.0L);
  for (int l = start; l >= 1; --l) {
    // j_{l-1} = (2l+1)/x j_l - j_{l+1}
    const long double jm = (2 * l + 1) / x * jc - jp;
    jp = jc;
    jc = jm;
    if (l - 1 <= lmax) tmp[l - 1] = jc;
    norm += (2 * (l - 1) + 1) * jc * jc;
    if (std::fabs((double)jc) > 1e200) {   // rescale to stay in range
      jp *= 1e-200L;
      jc *= 1e-200L;
      norm *= 1e-400L;
      for (auto& v : tmp) v *= 1e-200L;
    }
  }
  // sum_{l >= 0} (2l+1) j_l^2 = 1 fixes the scale; the sign follows j_0 or j_1,
  // whichever is larger in magnitude
  const long double scale = 1.0L / std::sqrt(norm);
  const long double j0 = std::sin(x) / x, j1 = std::sin(x) / (x * x) - std::cos(x) / x;
  long double sgn = 1.0L;
  if (std::fabs(j0) >= std::fabs(j1)) sgn = (j0 < 0) == (tmp[0] < 0) ? 1.0L : -1.0L;
  else if (lmax >= 1) sgn = (j1 < 0) == (tmp[1] < 0) ? 1.0L : -1.0L;
  for (int l = 0; l <= lmax; ++l) j[l] = sgn * scale * tmp[l];
}

void fh_cheb_matrix(int mmax, std::vector<long double>& M) {
  // discrete orthogonality of T_k at K > mmax Chebyshev-Gauss nodes is exact
  // for polynomials of degree < 2K - mmax: a_k = (2 - [k = 0]) / K sum_j p(u_j) T_k(u_j)
  const int K = mmax + 8;
  const long double pi = 3.141592653589793238462643383279502884L;
  M.assign((size_t)mmax * mmax, 0.0L);
  for (int j = 0; j < K; ++j) {
    const long double th = pi * (j + 0.5L) / K, u = cosl(th);
    long double q0 = 0.0L, q1 = 1.0L;   // Q_{m-1}, Q_m
    for (int m = 0; m < mmax; ++m) {
      if (m > 0) {
        const long double q2 = (fh_rec_A(m) * u + fh_rec_B(m)) * q1 - fh_rec_C(m) * q0;
        q0 = q1;
        q1 = q2;
      }
      for (int k = 0; k <= m; ++k) M[(size_t)k * mmax + m] += q1 * cosl(k * th) * (k == 0 ? 1.0L : 2.0L) / K;
    }
  }
}

}  // namespace bzq
