// Host-side series of the angular weight used by plans that evaluate their
// weights on the fly instead of storing a table.
//
// The weight of eq. FF depends on k only through r = a |k| and t = k.sigma / |k|.
// Expanding the plane wave in Legendre polynomials and integrating b over the
// sphere term by term (the Funk-Hecke formula) gives
//
//   Re(e^{-ix} F) = sum_{l even} (2l+1) (-1)^{l/2} mu_l j_l(r) P_l(t),
//   mu_l = 2 pi \int_{-1}^{1} b(u) (P_l(u) - 1) du
//        = 4 pi c \int_0^1 tau^{-s} (1-tau)^{-r} (P_l(1 - 2 tau) - 1) / tau d tau,
//
// for b = c tau^{-1-s} (1-tau)^{-r}, tau = sin^2(theta/2).  The "- 1" of eq. FF
// is what makes mu_l finite for the non-cutoff kernels (s < 1); (P_l - 1)/tau
// is a polynomial of degree l - 1, so an n-point Gauss-Jacobi rule with
// 2n >= l gives mu_l exactly.  The series converges like j_l(r) for l > r.
#pragma once
#include <vector>

namespace bzq {

// Highest even l kept for arguments up to r: the truncation error of the
// series is below 1e-13 relative for r <= 60.
int fh_lmax(double r);

// mu_l for even l = 0, 2, .., lmax (mu_0 = 0) into mu[l/2]; false if the
// Gauss-Jacobi rule cannot be built (s >= 1 or r >= 1).
bool fh_moments(int lmax, double c, double s, double r, std::vector<long double>& mu);

// Spherical Bessel functions j_l(x), l = 0..lmax (x >= 0), by Miller's
// backward recurrence normalised with sum_l (2l+1) j_l(x)^2 = 1.
void fh_sph_bessel(int lmax, long double x, std::vector<long double>& j);

// Connection matrix from Q_m(u) = P_{2m}(t) (u = 2t^2 - 1, below) to Chebyshev
// polynomials: Q_m(u) = sum_{k <= m} M[k * mmax + m] T_k(u), k, m < mmax.
// A series in Q_m becomes sum_k d_k T_k(u) with d = M c, which Clenshaw's rule
// sums with the same constant recurrence (2u) at every term.
void fh_cheb_matrix(int mmax, std::vector<long double>& M);

// Three-term recurrence of Q_m(u) = P_{2m}(t), u = 2 t^2 - 1 (the Jacobi
// polynomials P_m^{(0,-1/2)}):  Q_m = (A_m u + B_m) Q_{m-1} - C_m Q_{m-2},
// m >= 1 (C_1 = 0).  With g = 2m - 1/2 and D = 2m (m - 1/2)(g - 2):
// A_m = (g-1) g (g-2) / D, B_m = -(g-1) / (4D), C_m = 2 (m-1)(m-3/2) g / D.
// constexpr, so that the device kernel sees them as immediates.
constexpr double fh_rec_D(int m) { return 2.0 * m * (m - 0.5) * (2.0 * m - 2.5); }
constexpr double fh_rec_A(int m) { return (2.0 * m - 1.5) * (2.0 * m - 0.5) * (2.0 * m - 2.5) / fh_rec_D(m); }
constexpr double fh_rec_B(int m) { return -(2.0 * m - 1.5) * 0.25 / fh_rec_D(m); }
constexpr double fh_rec_C(int m) { return m <= 1 ? 0.0 : 2.0 * (m - 1) * (m - 1.5) * (2.0 * m - 0.5) / fh_rec_D(m); }

}  // namespace bzq
